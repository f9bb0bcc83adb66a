// C ABI of the FDTD gradient library: validation, buffer layout, the host time
// loops that sequence the kernels, the codec entry point and per-kernel timing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fdtd.h"
#include "march.h"

using namespace fdtd;

// Workspace of fdtd_forward_noalloc: one file-scope device array, which every device
// the library runs on holds at its own address until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a stand-in): it
// asks for the current device's address once (scratch_for_current_device) and uses that.
static __device__ __align__(256) unsigned char scratch[FDTD_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// Tuning override for tile sizes (read once per call; defaults otherwise).
#ifndef FDTD_FIELD_PAD
#define FDTD_FIELD_PAD 1056
#endif
// Floats between consecutive field components (cells rounded up to a 128-byte line,
// plus FDTD_FIELD_PAD floats).
int64_t field_stride(int64_t cells) { return ((cells + 31) / 32) * 32 + FDTD_FIELD_PAD; }

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    return h;
}

struct Plan {
    Grid g;
    Tiling fwd;            // forward sweep: the whole grid
    Tiling fwd2;           // two-step forward sweep: the whole grid
    int fwd_steps = 1;     // forward steps per sweep (1, or 2 where the two-step sweep applies)
    Tiling adj;            // adjoint sweep: the whole grid
    Tiling rev;            // primal reversal: the interior plus its shell
    Tiling rev2;           // two-step primal reversal: the interior
    int rev_steps = 1;     // reverse primal steps per sweep (1, or 2 where the two-step sweep applies)
    int box_o[3], box_n[3];
    int rev_x0;                    // x origin of the primal-reversal tiles (128-byte aligned)
    fdtd_store_info_t info;
    uint64_t ws_coef = 0, ws_profile = 0, ws_partials = 0, ws_staging = 0, ws_fields = 0;
    uint64_t ws_order_fwd = 0, ws_order_adj = 0, ws_order_fwd2 = 0;   // tile-order tables
    uint64_t ws_order_rev = 0, ws_order_rev2 = 0;
    uint64_t ws_mid = 0;           // intermediate recorder values of a two-step sweep (one kept step, FP32)
    uint64_t ws_stash = 0;         // a two-step reversal's inputs of its second step's seed and gradient
    uint64_t psi_floats = 0;
    int per_step = 0;
    int64_t src_volume = 0;
    int64_t msrc_volume = 0;       // 0: no magnetic current
    uint64_t ws_mprofile = 0;
    float coef[12 * FDTD_MAX_PML];   // 12 P used
    uint64_t hash = 0;
};

bool box_inside_interior(const int32_t lo[3], const int32_t hi[3], const int n[3], int P) {
    for (int d = 0; d < 3; ++d)
        if (lo[d] < P || hi[d] > n[d] - P || lo[d] >= hi[d]) return false;
    return true;
}

// CPML tables indexed by the slab coordinate i' in [0, 2P).  Depth from the
// interior boundary: E nodes (x = i) and H nodes (x = i + 1/2); the low slab
// has i' = i, the high slab i' = i - (n - 2P), so the depth depends on i' only.
void cpml_tables(const fdtd_problem_t* p, double dt, float* coef) {
    const int P = p->pml;
    std::fill(coef, coef + 12 * (size_t)P, 0.0f);
    const double m = p->pml_order;
    const double sig_max = p->pml_sigma_scale * 0.8 * (m + 1.0);
    for (int node = 0; node < 2; ++node) {
        for (int s = 0; s < 2 * P; ++s) {
            double depth;
            if (node == 0) depth = s < P ? (double)(P - s) : (double)(s - P) + 0.5;
            else depth = s < P ? (double)(P - s) - 0.5 : (double)(s - P) + 1.0;
            const double rho = depth / P;
            const double rm = std::pow(rho, m);
            const double sigma = sig_max * rm;
            const double kappa = 1.0 + (p->pml_kappa_max - 1.0) * rm;
            const double alpha = p->pml_alpha_max * (1.0 - rho);
            const double b = std::exp(-(sigma / kappa + alpha) * dt);
            const double a = sigma > 0.0 ? sigma * (b - 1.0) / (sigma * kappa + kappa * kappa * alpha) : 0.0;
            float* base = coef + (size_t)node * 6 * P;
            base[s] = (float)b;
            base[2 * P + s] = (float)a;
            base[4 * P + s] = (float)(1.0 / kappa);
        }
    }
}

int make_plan(const fdtd_problem_t* p, const fdtd_store_cfg_t* cfg, Plan* pl) {
    if (!p || !cfg) return fail(FDTD_EINVAL, "problem and store config must not be NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(FDTD_EINVAL, "grid extents must be >= 1 (got %d x %d x %d)", p->nx, p->ny, p->nz);
    // kernels address the six field components as one buffer with 32-bit byte offsets below 2^31
    if (p->ny > 4 * 65535 || p->nz > 65535 || 24 * field_stride((int64_t)p->nx * p->ny * p->nz) >= ((int64_t)1 << 31))
        return fail(FDTD_EINVAL, "grid too large: 24 * field stride must stay below 2^31");
    if (p->steps < 1) return fail(FDTD_EINVAL, "steps must be >= 1 (got %d)", p->steps);
    if (p->pml < 0 || p->pml > FDTD_MAX_PML) return fail(FDTD_EINVAL, "pml must be in [0, %d]", FDTD_MAX_PML);
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int d = 0; d < 3; ++d)
        if (2 * p->pml >= n[d]) return fail(FDTD_EINVAL, "2 * pml must be smaller than every extent");
    if (p->boundary != 0 && p->boundary != 1) return fail(FDTD_EINVAL, "boundary must be 0 or 1");
    if (p->boundary == 1 && p->pml != 0) return fail(FDTD_EINVAL, "a periodic grid has no PML (pml must be 0)");
    if (!(std::isfinite(p->courant) && p->courant > 0.0 && p->courant <= 1.0))
        return fail(FDTD_ECFL, "Courant number %g outside (0, 1]", p->courant);
    if (p->pml_order < 1 || !(p->pml_sigma_scale >= 0.0) || !(p->pml_kappa_max >= 1.0) ||
        !(p->pml_alpha_max >= 0.0) || !std::isfinite(p->pml_sigma_scale) || !std::isfinite(p->pml_kappa_max) ||
        !std::isfinite(p->pml_alpha_max))
        return fail(FDTD_EINVAL, "invalid PML grading parameters");
    if (p->src_comp < 0 || p->src_comp > 2) return fail(FDTD_EINVAL, "src_comp must be 0, 1 or 2");
    if (p->loss < 0 || p->loss > 3) return fail(FDTD_EINVAL, "loss must be 0 (|E|^2) or 1, 2, 3 (flux along x, y, z)");
    if (!p->src_wave || !p->src_profile) return fail(FDTD_EINVAL, "source signal and profile must not be NULL");
    if (!box_inside_interior(p->src_lo, p->src_hi, n, p->pml))
        return fail(FDTD_EREGION, "source box must be non-empty and inside the interior");
    const bool has_m = p->msrc_hi[0] > p->msrc_lo[0] && p->msrc_hi[1] > p->msrc_lo[1] && p->msrc_hi[2] > p->msrc_lo[2];
    if (has_m) {
        if (p->msrc_comp < 0 || p->msrc_comp > 2) return fail(FDTD_EINVAL, "msrc_comp must be 0, 1 or 2");
        if (!p->msrc_wave || !p->msrc_profile)
            return fail(FDTD_EINVAL, "magnetic current signal and profile must not be NULL");
        if (!box_inside_interior(p->msrc_lo, p->msrc_hi, n, p->pml))
            return fail(FDTD_EREGION, "magnetic current box must be inside the interior");
    }
    if (!box_inside_interior(p->det_lo, p->det_hi, n, p->pml))
        return fail(FDTD_EREGION, "detector box must be non-empty and inside the interior");
    if (!box_inside_interior(p->des_lo, p->des_hi, n, p->pml))
        return fail(FDTD_EREGION, "design box must be non-empty and inside the interior");
    if (cfg->dtype < FDTD_STORE_FP32 || cfg->dtype > FDTD_STORE_FP8_E4M3FN)
        return fail(FDTD_ESTORE, "unknown storage type %d", cfg->dtype);
    if (cfg->k < 1) return fail(FDTD_ESTORE, "subsampling k must be >= 1 (got %d)", cfg->k);
    if (cfg->interp != 0 && cfg->interp != FDTD_INTERP_LINEAR && cfg->interp != FDTD_INTERP_CUBIC)
        return fail(FDTD_ESTORE, "interp must be 0 or 1 (linear) or 3 (cubic) (got %d)", cfg->interp);

    const int P = p->pml;
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const double dt = p->courant / std::sqrt(3.0);   // Eq. 1 with dx = c = 1
    Grid& g = pl->g;
    std::memset(&g, 0, sizeof g);
    g.nx = p->nx; g.ny = p->ny; g.nz = p->nz; g.P = P;
    g.periodic = p->boundary;
    g.mx = p->nx - 2 * P; g.my = p->ny - 2 * P; g.mz = p->nz - 2 * P;
    g.N = field_stride(N);
    g.dt = (float)dt;
    g.slab[0] = 2LL * P * p->ny * p->nz;
    g.slab[1] = 2LL * P * p->nx * p->nz;
    g.slab[2] = 2LL * P * p->nx * p->ny;
    g.psi_off[0] = 0;
    g.psi_off[1] = 4 * g.slab[0];
    g.psi_off[2] = 4 * (g.slab[0] + g.slab[1]);
    g.psi_total = 4 * (g.slab[0] + g.slab[1] + g.slab[2]);
    if (8 * (int64_t)g.psi_total >= ((int64_t)1 << 31))
        return fail(FDTD_EINVAL, "PML too large: the two copies of the auxiliaries must stay below 2 GiB");
    g.src_comp = p->src_comp;
    g.loss = p->loss;
    g.msrc_comp = has_m ? p->msrc_comp : 0;
    for (int d = 0; d < 3; ++d) {
        g.msrc_lo[d] = has_m ? p->msrc_lo[d] : 0;
        g.msrc_hi[d] = has_m ? p->msrc_hi[d] : 0;
    }
    for (int d = 0; d < 3; ++d) {
        g.src_lo[d] = p->src_lo[d]; g.src_hi[d] = p->src_hi[d];
        g.det_lo[d] = p->det_lo[d]; g.det_hi[d] = p->det_hi[d];
        g.des_lo[d] = p->des_lo[d]; g.des_hi[d] = p->des_hi[d];
    }
    g.dtype = cfg->dtype;
    const int64_t vps = P > 0 ? 4LL * ((int64_t)g.my * g.mz + (int64_t)g.mx * g.mz + (int64_t)g.mx * g.my) : 0;
    g.vps = vps;
    const uint64_t vbytes = (uint64_t)storage_bytes(cfg->dtype);
    const uint64_t slices = ((uint64_t)p->steps + cfg->k - 1) / cfg->k;
    g.slice_stride = (long long)align_up(vps * vbytes, 256);
    g.scale_off = (long long)(slices * (uint64_t)g.slice_stride);
    g.dbx0 = p->det_lo[0] / BX; g.dnbx = (p->det_hi[0] - 1) / BX - g.dbx0 + 1;
    g.dby0 = p->det_lo[1] / BY; g.dnby = (p->det_hi[1] - 1) / BY - g.dby0 + 1;
    g.dbz0 = p->det_lo[2];      g.dnbz = p->det_hi[2] - p->det_lo[2];
    Tiling& t = pl->fwd;
    // 8-row tiles (fewer re-read ring rows per cell) unless the grid has fewer 8-row
    // tiles than compute units; measured: 256x256x128 forward 126.4 -> 123.2 us, adjoint
    // 142.4 -> 139.9, 512x512x256 adjoint 978 -> 962, 128^3 forward 28.2 -> 27.8, but
    // 32^3 (16 tiles) forward 17.2 -> 19.9
    const long long tiles8 = (long long)((p->nx + TX - 1) / TX) * ((p->ny + 7) / 8) * ((p->nz + 7) / 8);
    const int ty_default = tiles8 >= 256 ? 8 : 4;
    t.ty = env_int("FDTD_TILE_Y", ty_default) == 8 ? 8 : 4;
    t.cz = env_int("FDTD_TILE_Z", 8) == 4 ? 4 : 8;
    t.ntx = (p->nx + TX - 1) / TX;
    t.nty = (p->ny + t.ty - 1) / t.ty;
    t.ntz = (p->nz + t.cz - 1) / t.cz;
    t.count = t.ntx * t.nty * t.ntz;
    t.dtx0 = p->det_lo[0] / TX; t.dntx = (p->det_hi[0] - 1) / TX - t.dtx0 + 1;
    t.dty0 = p->det_lo[1] / t.ty; t.dnty = (p->det_hi[1] - 1) / t.ty - t.dty0 + 1;
    t.dtz0 = p->det_lo[2] / t.cz; t.dntz = (p->det_hi[2] - 1) / t.cz - t.dtz0 + 1;
    pl->per_step = t.dntx * t.dnty * t.dntz;
    t.order = nullptr;
    {
        // two forward steps per sweep: tiles of W2 columns, 12 rows, 16 (or 8) planes; not
        // with a magnetic-current sheet (the single-step sweep carries it).  Measured at
        // 512x512x256: 12x16 1620 us per launch, 12x8 1815, 8x16 1907 (8 rows: 146 registers,
        // one 12-wave block per compute unit).
        Tiling& t2 = pl->fwd2;
        t2 = t;
        t2.ty = 12;
        t2.cz = env_int("FDTD_FWD2_TILE_Z", 16) == 8 ? 8 : 16;
        t2.ntx = (p->nx + W2 - 1) / W2;
        t2.nty = (p->ny + t2.ty - 1) / t2.ty;
        t2.ntz = (p->nz + t2.cz - 1) / t2.cz;
        t2.count = t2.ntx * t2.nty * t2.ntz;
        t2.dtx0 = p->det_lo[0] / W2; t2.dntx = (p->det_hi[0] - 1) / W2 - t2.dtx0 + 1;
        t2.dty0 = p->det_lo[1] / t2.ty; t2.dnty = (p->det_hi[1] - 1) / t2.ty - t2.dty0 + 1;
        t2.dtz0 = p->det_lo[2] / t2.cz; t2.dntz = (p->det_hi[2] - 1) / t2.cz - t2.dtz0 + 1;
        t2.order = nullptr;
        // Two steps per sweep where at least half of the two-step tiles reach no PML slab.
        // The sweep recomputes a two-cell halo (about 1.4x the arithmetic of two single
        // steps), which the halved traffic pays for in interior tiles; tiles that carry
        // PML auxiliaries cost about twice as much and hold the kernel's register budget.
        // Measured: 512x512x256 (53 % interior tiles) forward 928 -> 810 us per step;
        // 256x256x128 (39 %) 129.5 -> 136; 128^3 (none) 32.5 -> 55.
        // FDTD_FWD_STEPS=1 or 2 overrides the choice.
        int interior = 0;
        for (int L = 0; L < t2.count; ++L) {
            const int a = (L % t2.ntx) * W2, j0 = ((L / t2.ntx) % t2.nty) * t2.ty, k0 = (L / (t2.ntx * t2.nty)) * t2.cz;
            if (slab_class(g, a - 2, a + TX - 3, j0 - 2, j0 + t2.ty + 1, k0 - 2, k0 + t2.cz) == 0) ++interior;
        }
        const int want = env_int("FDTD_FWD_STEPS", 0);
        const bool two = want == 2 || (want != 1 && 2LL * interior >= t2.count);
        pl->fwd_steps = (!has_m && two) ? 2 : 1;
        // room for either sweep's detector tiles (the unused entries are zeroed by the call)
        pl->per_step = std::max(pl->per_step, t2.dntx * t2.dnty * t2.dntz);
    }
    for (int d = 0; d < 3; ++d) {
        pl->box_o[d] = P > 0 ? P - 1 : 0;
        pl->box_n[d] = P > 0 ? n[d] - 2 * P + 2 : n[d];
    }
    Tiling& a = pl->adj;
    a = t;
    a.ty = env_int("FDTD_ADJ_TILE_Y", ty_default) == 8 ? 8 : 4;
    a.cz = env_int("FDTD_ADJ_TILE_Z", 8) == 4 ? 4 : 8;
    a.nty = (p->ny + a.ty - 1) / a.ty;
    a.ntz = (p->nz + a.cz - 1) / a.cz;
    a.count = a.ntx * a.nty * a.ntz;
    Tiling& r = pl->rev;
    r = t;
    pl->rev_x0 = pl->box_o[0] & ~31;
    r.ntx = (pl->box_o[0] + pl->box_n[0] - pl->rev_x0 + TX - 1) / TX;
    {
        // Shape of the reversal's tiles: 4 rows and, among 4, 5 and 6 planes, the depth whose
        // tile count fills most of one round (five 4-wave workgroups on each of 256 compute
        // units) when some depth fits in a round, else 6 (the least re-read z halo); 8 x 8
        // where the 4 x 6 tiling takes more than eight rounds.  Measured at 128^3 (one round
        // at depth 5: 22.0 -> 20.6 us), 256x256x128 (3.3 rounds: 4 x 6 88.2 us, 8 x 8 88.4)
        // and 512x512x256 (29 rounds: 716 -> 696 us with 8 x 8).
        const long long slots = 5 * 256, cols = (long long)r.ntx * ((pl->box_n[1] + 3) / 4);
        int pick = 6;
        long long best = 0;
        for (int cz = 4; cz <= 6; ++cz) {
            const long long n = cols * ((pl->box_n[2] + cz - 1) / cz);
            if (n <= slots && n > best) { best = n; pick = cz; }
        }
        const bool big = cols * ((pl->box_n[2] + 5) / 6) > 8 * slots;
        r.ty = env_int("FDTD_REV_TILE_Y", big ? 8 : 4) == 8 ? 8 : 4;
        const int cz = env_int("FDTD_REV_TILE_Z", r.ty == 4 ? pick : (big ? 8 : 4));
        r.cz = (cz == 8 || (r.ty == 4 && (cz == 5 || cz == 6))) ? cz : 4;
    }
    r.nty = (pl->box_n[1] + r.ty - 1) / r.ty;
    {
        // two reverse steps per sweep over the interior (60 x 12 columns, 16 planes); not with
        // a magnetic-current sheet, and not on a periodic grid with PML
        Tiling& r2 = pl->rev2;
        r2 = t;
        r2.ty = 12;
        r2.cz = env_int("FDTD_REV2_TILE_Z", 16) == 8 ? 8 : 16;
        const int mxi = n[0] - 2 * P, myi = n[1] - 2 * P, mzi = n[2] - 2 * P;
        r2.ntx = (mxi + W2 - 1) / W2;
        r2.nty = (myi + r2.ty - 1) / r2.ty;
        r2.ntz = (mzi + r2.cz - 1) / r2.cz;
        r2.count = r2.ntx * r2.nty * r2.ntz;
        r2.order = nullptr;
        // Chosen where its launch is at least eight rounds of one 16-wave block per compute
        // unit: the reversal is bound by issue and latency more than by HBM, so the halved
        // traffic pays for the recomputed halo only when the chip stays full.  Measured:
        // 512x512x256 (4480 blocks) 694 -> 627 us per step; 256x256x128 (560) 78 -> 113;
        // 128^3 (126) 19 -> 39.  FDTD_REV_STEPS=1 or 2 overrides the choice.
        const bool able = !has_m && !(p->boundary && P > 0) && mxi > 0 && myi > 0 && mzi > 0;
        const int want = env_int("FDTD_REV_STEPS", 0);
        pl->rev_steps = (able && (want == 2 || (want != 1 && r2.count >= 8 * 256))) ? 2 : 1;
    }
    r.ntz = (pl->box_n[2] + r.cz - 1) / r.cz;
    r.count = r.ntx * r.nty * r.ntz;
    pl->psi_floats = (uint64_t)g.psi_total;
    pl->src_volume = (int64_t)(p->src_hi[0] - p->src_lo[0]) * (p->src_hi[1] - p->src_lo[1]) *
                     (p->src_hi[2] - p->src_lo[2]);

    fdtd_store_info_t& in = pl->info;
    std::memset(&in, 0, sizeof in);
    in.cells = (uint64_t)N;
    in.slices = slices;
    in.values_per_slice = (uint64_t)vps;
    in.payload_bytes = slices * (uint64_t)vps * vbytes;
    in.scale_bytes = cfg->dtype == FDTD_STORE_FP8_E4M3_SCALED ? slices * 12 * 4 : 0;
    in.store_bytes = std::max<uint64_t>(256, (uint64_t)g.scale_off + align_up(in.scale_bytes, 256));
    in.fields_bytes = 6ull * (uint64_t)g.N * 4;
    in.psi_bytes = std::max<uint64_t>(256, 2 * pl->psi_floats * 4);
    in.adj_psi_bytes = std::max<uint64_t>(512, 2 * pl->psi_floats * 4);
    pl->ws_coef = 0;
    pl->ws_profile = align_up(12ull * P * 4, 256);
    pl->msrc_volume = has_m ? (int64_t)(p->msrc_hi[0] - p->msrc_lo[0]) * (p->msrc_hi[1] - p->msrc_lo[1]) *
                                  (p->msrc_hi[2] - p->msrc_lo[2]) : 0;
    pl->ws_mprofile = pl->ws_profile + align_up((uint64_t)pl->src_volume * 4, 256);
    pl->ws_partials = pl->ws_mprofile + align_up((uint64_t)pl->msrc_volume * 4, 256);
    pl->ws_staging = pl->ws_partials + align_up((uint64_t)p->steps * pl->per_step * 8, 256);
    const uint64_t staging =
        cfg->dtype == FDTD_STORE_FP8_E4M3_SCALED ? align_up((uint64_t)rec_quant_scratch_floats(g) * 4, 256) : 0;
    pl->ws_order_fwd = pl->ws_staging + staging;
    pl->ws_order_adj = pl->ws_order_fwd + align_up(4ull * pl->fwd.count, 256);
    // the two-step sweep's order table and intermediate recorder values are reserved whether
    // or not it is chosen, so that the size store_config reports does not depend on the choice
    pl->ws_order_fwd2 = pl->ws_order_adj + align_up(4ull * pl->adj.count, 256);
    pl->ws_order_rev = pl->ws_order_fwd2 + align_up(4ull * pl->fwd2.count, 256);
    pl->ws_order_rev2 = pl->ws_order_rev + align_up(4ull * pl->rev.count, 256);
    pl->ws_mid = pl->ws_order_rev2 + align_up(4ull * pl->rev2.count, 256);
    pl->ws_stash = pl->ws_mid + align_up((uint64_t)g.vps * 4, 256);
    {
        const uint64_t ndet = (uint64_t)(p->det_hi[0] - p->det_lo[0]) * (p->det_hi[1] - p->det_lo[1]) *
                              (p->det_hi[2] - p->det_lo[2]);
        const uint64_t ndes = (uint64_t)(p->des_hi[0] - p->des_lo[0]) * (p->des_hi[1] - p->des_lo[1]) *
                              (p->des_hi[2] - p->des_lo[2]);
        pl->ws_fields = pl->ws_stash + align_up((6 * ndet + 4 * ndes) * 4, 256);
    }
    // second primal and second adjoint field buffers (ping-pong)
    in.workspace_bytes = pl->ws_fields + 2 * in.fields_bytes;
    in.design_cells = (uint64_t)(p->des_hi[0] - p->des_lo[0]) * (p->des_hi[1] - p->des_lo[1]) *
                      (p->des_hi[2] - p->des_lo[2]);

    cpml_tables(p, dt, pl->coef);

    uint64_t h = 1469598103934665603ull;
    const int32_t ints[] = {p->nx, p->ny, p->nz, p->pml, p->steps, p->boundary, p->pml_order, p->src_comp,
                            p->src_lo[0], p->src_lo[1], p->src_lo[2], p->src_hi[0], p->src_hi[1], p->src_hi[2],
                            p->det_lo[0], p->det_lo[1], p->det_lo[2], p->det_hi[0], p->det_hi[1], p->det_hi[2],
                            p->des_lo[0], p->des_lo[1], p->des_lo[2], p->des_hi[0], p->des_hi[1], p->des_hi[2], p->loss};
    const double dbl[] = {p->courant, p->pml_sigma_scale, p->pml_kappa_max, p->pml_alpha_max};
    h = fnv1a(h, ints, sizeof ints);
    h = fnv1a(h, dbl, sizeof dbl);
    h = fnv1a(h, p->src_wave, (size_t)p->steps * 4);
    h = fnv1a(h, p->src_profile, (size_t)pl->src_volume * 4);
    if (pl->msrc_volume > 0) {
        const int32_t mi[] = {p->msrc_comp, p->msrc_lo[0], p->msrc_lo[1], p->msrc_lo[2],
                              p->msrc_hi[0], p->msrc_hi[1], p->msrc_hi[2]};
        h = fnv1a(h, mi, sizeof mi);
        h = fnv1a(h, p->msrc_wave, (size_t)p->steps * 4);
        h = fnv1a(h, p->msrc_profile, (size_t)pl->msrc_volume * 4);
    }
    pl->hash = h;
    return FDTD_OK;
}

// Launch order of a sweep's tiles (the device computes each tile's class again from its
// coordinates; the order only decides where and beside what each block runs).  The
// position p of a block goes to XCD p / (count / 8) (logical_tile), so the order is
// dealt out in eight equal chunks: every chunk gets an eighth of each class's tiles
// (classes differ in cost; in plain x-y-z order the z-slab tiles, the costliest, would
// all land on the first and last XCD), and within a chunk the tiles come class by class,
// each class in x-y-z order (neighbouring tiles share halo lines in that XCD's L2, and
// the blocks running side by side mostly share one class's code).
// A forward launch (one or two steps per sweep) of more than two rounds of the chip
// (a compute unit holds two 8-wave, four 4-wave or one 16-wave workgroup), and an
// adjoint launch of at least eight, is ordered by octants instead: the tile grid halved
// along each axis, octant after octant (an XCD's chunk is then one octant when the
// halves are equal), costliest class first within an octant.  Every octant holds one
// PML side of each axis, so the chunks carry equal work on a symmetric grid.  Measured:
// 512x512x256 adjoint 952 -> 915 us (32 rounds), two-step forward 1622 -> 1606 us;
// 256x256x128 (4 rounds) forward 124.2 -> 121.4 but adjoint 140.5 -> 141.7; launches
// of one round (128^3) ran 15-20 % slower that way.
// The primal reversal's tiles (one or two steps per sweep) all run one code path; by
// default they go in x-y-z order dealt out in chunks (no table).  The one-step reversal
// goes by octants where its launch takes more than two rounds: 256x256x128 reversal
// 87.4 -> 84.2 us (the adjoint after it 140.4 -> 141.7), while 128^3 (one round) went
// 19.0 -> 21.6.  The two-step reversal keeps its natural order (512x512x256 by
// octants: 1246 -> 1379 us).
// FDTD_TILE_ORDER=1 (classes dealt out, or no table) or 2 (octants) overrides the choice.
// which: 0 forward, 1 adjoint, 2 two-step forward, 3 reversal, 4 two-step reversal; an
// empty table means the reversal keeps its natural order.
void tile_order(const Plan& pl, int which, std::vector<int32_t>& out) {
    const Tiling& t = which == 0 ? pl.fwd
                      : which == 1 ? pl.adj
                      : which == 2 ? pl.fwd2
                      : which == 3 ? pl.rev
                                   : pl.rev2;
    std::vector<int32_t> cls((size_t)t.count);
    int counts[8] = {0};
    for (int L = 0; L < t.count; ++L) {
        const int tix = L % t.ntx, tiy = (L / t.ntx) % t.nty, tiz = L / (t.ntx * t.nty);
        const int j0 = tiy * t.ty, k0 = tiz * t.cz;
        int c = 0;
        if (which >= 3) {
            // one code path for every tile
        } else if (which == 2) {
            const int a = tix * W2;   // the two-step tile reads two cells around its own
            c = slab_class(pl.g, a - 2, a + TX - 3, j0 - 2, j0 + t.ty + 1, k0 - 2, k0 + t.cz);
        } else {
            const int i0 = tix * TX;
            c = slab_class(pl.g, i0 - 1, i0 + TX, j0 - 1, j0 + t.ty, k0 - 1, k0 + t.cz);
        }
        cls[(size_t)L] = c;
        ++counts[c];
    }
    out.clear();
    out.reserve((size_t)t.count);
    // twice the rounds of the chip the launch takes, rounded down (16 waves per compute unit)
    const long long rounds_x2 = (which == 2 || which == 4) ? 2LL * t.count / 256 : 2LL * t.count * t.ty / (16 * 256);
    const int want = env_int("FDTD_TILE_ORDER", 0);
    const bool by_rounds = which == 4 ? false : (which == 1 ? rounds_x2 >= 16 : rounds_x2 > 4);
    if (want == 2 || (want != 1 && by_rounds)) {
        const int n[3] = {t.ntx, t.nty, t.ntz};
        const int h[3] = {(t.ntx + 1) / 2, (t.nty + 1) / 2, (t.ntz + 1) / 2};
        std::vector<int32_t> part;
        for (int o = 0; o < 8; ++o) {
            int lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                const bool up = ((o >> d) & 1) != 0;
                lo[d] = up ? h[d] : 0;
                hi[d] = up ? n[d] : h[d];
            }
            part.clear();
            for (int z = lo[2]; z < hi[2]; ++z)
                for (int y = lo[1]; y < hi[1]; ++y)
                    for (int x = lo[0]; x < hi[0]; ++x) part.push_back(x + t.ntx * (y + t.nty * z));
            std::stable_sort(part.begin(), part.end(),
                             [&](int32_t a, int32_t b) { return cls[(size_t)a] > cls[(size_t)b]; });
            out.insert(out.end(), part.begin(), part.end());
        }
        return;
    }
    if (which >= 3) return;   // natural order
    std::vector<int32_t> by_class[8];
    for (int c = 0; c < 8; ++c) by_class[c].reserve((size_t)counts[c]);
    for (int L = 0; L < t.count; ++L) by_class[cls[(size_t)L]].push_back(L);
    // single-step sweeps: the costliest classes first (class 7, all three slabs, down to
    // class 0), so that the chunk's last blocks are cheap ones and its tail is short
    // (256x256x128: forward 131.8 -> 126.2 us, adjoint 147.7 -> 142.2); the two-step
    // sweep, whose launch is a few rounds of large blocks, measured 1 % slower that way
    const bool costly_first = which != 2;
    for (int x = 0; x < 8; ++x)
        for (int i = 0; i < 8; ++i) {
            const int c = costly_first ? 7 - i : i;
            const size_t n = by_class[c].size(), lo = n * x / 8, hi = n * (x + 1) / 8;
            out.insert(out.end(), by_class[c].begin() + (long)lo, by_class[c].begin() + (long)hi);
        }
}

// The CPML coefficient table and the source profiles into the workspace, written by
// kernel launches that carry the values (so a captured graph holds them, and the
// call reads no host memory after it returns).  Both directions write them, so a
// backward call needs nothing that its forward left in the workspace.
void put_tables(const Plan& pl, const fdtd_problem_t* prob, char* ws, hipStream_t q) {
    launch_put((float*)(ws + pl.ws_coef), pl.coef, 12LL * pl.g.P, q);
    launch_put((float*)(ws + pl.ws_profile), prob->src_profile, pl.src_volume, q);
    if (pl.msrc_volume > 0) launch_put((float*)(ws + pl.ws_mprofile), prob->msrc_profile, pl.msrc_volume, q);
}

// Weights of the reinjection at reverse step n (kept steps T-1-j*k, j = 0 .. M-1, and the
// zero anchor at -1).  Linear: the two kept neighbours.  Cubic (interp 3): the Lagrange
// polynomial through the four consecutive nodes around n (times ascending: the anchor,
// then the kept steps), with n in the middle interval unless that runs past either end
// of the nodes; linear when there are fewer than four nodes.
Interp interp_for(int n, int T, int k, int interp) {
    Interp q;
    for (int t = 0; t < 4; ++t) { q.j[t] = -1; q.w[t] = 0.0f; }
    if ((T - 1 - n) % k == 0) {
        q.j[0] = (T - 1 - n) / k;
        q.w[0] = 1.0f;
        return q;
    }
    const int M = (T + k - 1) / k;                 // kept steps
    if (interp == FDTD_INTERP_CUBIC && M >= 3) {
        const int nmin = T - 1 - (M - 1) * k;      // earliest kept step
        auto node_time = [&](int i) { return i == 0 ? -1 : nmin + (i - 1) * k; };   // i = 0 .. M
        const int i = n < nmin ? 0 : 1 + (n - nmin) / k;                           // node_time(i) < n < node_time(i+1)
        const int s = std::min(std::max(i - 1, 0), M - 3);
        for (int a = 0; a < 4; ++a) {
            double w = 1.0;
            for (int b = 0; b < 4; ++b)
                if (b != a) w *= (double)(n - node_time(s + b)) / (double)(node_time(s + a) - node_time(s + b));
            q.j[a] = s + a == 0 ? -1 : M - (s + a);   // slice of the node (the anchor has none)
            q.w[a] = (float)w;
        }
        return q;
    }
    const int j1 = (T - 1 - n) / k;
    const int n1 = T - 1 - j1 * k;
    int n0 = n1 - k, j0 = j1 + 1;
    if (n0 < 0) { n0 = -1; j0 = -1; }
    const double w = (double)(n - n0) / (double)(n1 - n0);
    q.j[0] = j1; q.w[0] = (float)w;
    q.j[1] = j0; q.w[1] = (float)(1.0 - w);
    return q;
}

int check_hip(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FDTD_EHIP, "%s: %s", what, hipGetErrorString(e));
    return FDTD_OK;
}

// ---- per-kernel timing ------------------------------------------------------
const char* kKindNames[K_NUM_KINDS] = {"fill", "fwd_step", "rec_quant", "loss_final", "inject_shell",
                                       "prim_rev", "adj_step", "scale_grad", "codec", "put", "record", "fwd2_step",
                                       "prim_rev2", "rev_pending"};
constexpr size_t kMaxTimedLaunches = 1 << 16;

struct Timing {
    std::mutex mu;
    bool enabled = false;
    std::vector<hipEvent_t> pool;      // 2 events per timed launch
    std::vector<int> kinds;            // kind of each timed launch
    size_t used = 0;
} g_timing;

// ---- HIP-graph replay of the time loops ------------------------------------
// A call whose problem, configuration, buffers and device match an earlier one
// replays that call's launch sequence as one graph: the T-step loop is
// captured once (on an internal stream) and then launched on the caller's
// stream.  Per-kernel timing bypasses graphs.
struct GraphEntry {
    uint64_t key;
    hipGraphExec_t exec;
    hipEvent_t done;     // recorded after every launch: eviction waits for the last one
};
struct GraphCache {
    std::mutex mu;
    bool enabled = true;
    std::vector<GraphEntry> entries;   // most recent last
    hipStream_t capture[64] = {};      // per device
} g_graphs;
constexpr size_t kMaxGraphs = 16;

}  // namespace

namespace fdtd {
bool timing_acquire(int kind, hipEvent_t* start, hipEvent_t* stop) {
    if (!g_timing.enabled) return false;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (g_timing.used >= kMaxTimedLaunches) return false;
    while (g_timing.pool.size() < 2 * (g_timing.used + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return false;
        g_timing.pool.push_back(e);
    }
    *start = g_timing.pool[2 * g_timing.used];
    *stop = g_timing.pool[2 * g_timing.used + 1];
    if (g_timing.kinds.size() <= g_timing.used) g_timing.kinds.resize(g_timing.used + 1);
    g_timing.kinds[g_timing.used] = kind;
    ++g_timing.used;
    return true;
}
}  // namespace fdtd

namespace {

template <class Enqueue>
int run_sequence(uint64_t key, hipStream_t s, Enqueue&& enqueue, const char* what, bool allow_graph = true) {
    bool use_graph;
    {
        std::lock_guard<std::mutex> lk(g_graphs.mu);
        use_graph = allow_graph && g_graphs.enabled && !g_timing.enabled;
    }
    int dev = 0;
    if (use_graph && (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)) use_graph = false;
    if (!use_graph) {
        enqueue(s);
        return check_hip(what);
    }
    key = fnv1a(key, &dev, sizeof dev);
    std::lock_guard<std::mutex> lk(g_graphs.mu);
    for (GraphEntry& e : g_graphs.entries) {
        if (e.key == key) {
            if (hipGraphLaunch(e.exec, s) != hipSuccess || hipEventRecord(e.done, s) != hipSuccess)
                return fail(FDTD_EHIP, "%s: graph launch failed", what);
            return check_hip(what);
        }
    }
    hipStream_t& cap = g_graphs.capture[dev];
    if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        cap = nullptr;
        enqueue(s);
        return check_hip(what);
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(FDTD_EHIP, "%s: stream capture could not start", what);
    enqueue(cap);
    const hipError_t ce = hipStreamEndCapture(cap, &graph);
    if (ce != hipSuccess || !graph) return fail(FDTD_EHIP, "%s: stream capture failed: %s", what, hipGetErrorString(ce));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(FDTD_EHIP, "%s: graph instantiation failed: %s", what, hipGetErrorString(ie));
    hipEvent_t done = nullptr;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return fail(FDTD_EHIP, "%s: event creation failed", what);
    }
    if (g_graphs.entries.size() >= kMaxGraphs) {
        // the oldest graph may still run on some stream: wait for its last launch
        GraphEntry& old = g_graphs.entries.front();
        (void)hipEventSynchronize(old.done);
        (void)hipGraphExecDestroy(old.exec);
        (void)hipEventDestroy(old.done);
        g_graphs.entries.erase(g_graphs.entries.begin());
    }
    g_graphs.entries.push_back(GraphEntry{key, exec, done});
    if (hipGraphLaunch(exec, s) != hipSuccess || hipEventRecord(done, s) != hipSuccess)
        return fail(FDTD_EHIP, "%s: graph launch failed", what);
    return check_hip(what);
}

uint64_t call_key(const Plan& pl, int dir, const fdtd_store_cfg_t* cfg, std::initializer_list<const void*> ptrs) {
    uint64_t h = fnv1a(pl.hash, &dir, sizeof dir);
    h = fnv1a(h, cfg, sizeof *cfg);
    // the tile shapes and the launch-order choice (they can be changed between calls
    // through the environment)
    const int tiles[12] = {pl.fwd.ty, pl.fwd.cz, pl.adj.ty, pl.adj.cz, pl.rev.ty, pl.rev.cz,
                           pl.fwd2.ty, pl.fwd2.cz, pl.fwd_steps, pl.rev2.cz, pl.rev_steps,
                           env_int("FDTD_TILE_ORDER", 0)};
    h = fnv1a(h, tiles, sizeof tiles);
    for (const void* p : ptrs) h = fnv1a(h, &p, sizeof p);
    return h;
}

struct ScratchAddrs {
    std::mutex mu;
    void* ptr[64] = {};
} g_scratch;

int scratch_for_current_device(char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(FDTD_EHIP, "fdtd_forward_noalloc: no usable current device");
    std::lock_guard<std::mutex> lk(g_scratch.mu);
    if (!g_scratch.ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FDTD_EHIP, "fdtd_forward_noalloc: address of the scratch array on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch.ptr[dev] = p;
    }
    *out = (char*)g_scratch.ptr[dev];
    return FDTD_OK;
}

// The forward time loop on a workspace `ws` (the caller's, or the scratch array).
int forward_with(const Plan& pl, const fdtd_problem_t* prob, const fdtd_store_cfg_t* cfg, const float* eps,
                 float* fields, float* psi, void* store, char* ws, double* loss, double* loss_series,
                 fdtd_record_t* rec, hipStream_t s, bool allow_graph, const char* what) {
    Grid g = pl.g;
    // the caller's workspace holds the class-sorted tile order; the library's own array
    // (allow_graph false: no host allocation either) runs the tiles in x-y-z order
    Tiling fwd = pl.fwd, fwd2 = pl.fwd2;
    const bool two = pl.fwd_steps == 2;
    std::vector<int32_t> order, order2;
    fwd.order = fwd2.order = nullptr;
    if (allow_graph) {
        tile_order(pl, 0, order);
        fwd.order = (const int32_t*)(ws + pl.ws_order_fwd);
        if (two) {
            tile_order(pl, 2, order2);
            fwd2.order = (const int32_t*)(ws + pl.ws_order_fwd2);
        }
    }
    g.coef = (const float*)(ws + pl.ws_coef);
    g.src_profile = (const float*)(ws + pl.ws_profile);
    g.msrc_profile = (const float*)(ws + pl.ws_mprofile);
    double* partials = (double*)(ws + pl.ws_partials);
    float* staging = (float*)(ws + pl.ws_staging);

    const int64_t N = g.N;
    const int T = prob->steps, k = cfg->k;
    // Sweeps: one step per sweep, or (two-step mode) a single step first when T is odd,
    // then pairs.  Ping-pong field buffers; the parity of the sweep count picks the start
    // so that the final state lands in the caller's buffer.
    const int single = two ? (T & 1) : T;
    const int sweeps = two ? single + T / 2 : T;
    float* F[2] = {fields, (float*)(ws + pl.ws_fields)};
    const int start = sweeps & 1;
    const bool fp8 = cfg->dtype == FDTD_STORE_FP8_E4M3_SCALED && g.vps > 0;
    const float* wave = prob->src_wave;
    float* mid = two ? (float*)(ws + pl.ws_mid) : nullptr;
    auto mwave = [&](int n) { return pl.msrc_volume > 0 ? prob->msrc_wave[n] : 0.0f; };
    auto slice_of = [&](int n) { return ((T - 1 - n) % k == 0) ? (T - 1 - n) / k : -1; };
    auto record = [&](const float* E, bool e_mid, const float* H, bool h_mid, int slice, hipStream_t q) {
        launch_record(g, E, e_mid, H, h_mid, store, staging, slice, q);
        if (fp8) launch_rec_quant(g, staging, store, slice, q);
    };
    auto enqueue = [&](hipStream_t q) {
        put_tables(pl, prob, ws, q);
        if (fwd.order) launch_put(ws + pl.ws_order_fwd, order.data(), (long long)order.size(), q);
        if (fwd2.order) launch_put(ws + pl.ws_order_fwd2, order2.data(), (long long)order2.size(), q);
        launch_fill(F[start], 6 * N, 0.0f, q);
        launch_fill(psi, 2 * (long long)pl.psi_floats, 0.0f, q);
        // the two sweeps' tilings may meet the detector in different numbers of tiles
        launch_fill_f64(partials, (long long)T * pl.per_step, 0.0, q);
        int sw = 0, hc = 0, ec = 0;   // sweeps so far; PML copies holding the H-side and E-side auxiliaries
        // One step per sweep and a storage type written directly: trailing workgroups of the
        // sweeps record the kept steps, E^n of step n in sweep n (which reads it) and
        // H^{n+1/2} in sweep n+1 (which reads the buffer sweep n wrote); the last step's H
        // takes a launch of its own.  Otherwise the recorder launches after each kept step.
        const bool trail = !two && !fp8;
        auto slice_ptr = [&](int n) -> void* {
            const int sl = n >= 0 ? slice_of(n) : -1;
            return sl >= 0 ? (void*)((char*)store + (int64_t)sl * g.slice_stride) : nullptr;
        };
        for (int n = 0; n < single; ++n, ++sw) {
            const float* in = F[(start + sw) & 1];
            float* out = F[(start + sw + 1) & 1];
            const RecJob job{in, slice_ptr(n), slice_ptr(n - 1)};
            launch_fwd_step(g, fwd, in, out, psi, hc, eps, wave[n], mwave(n), partials + (int64_t)n * pl.per_step,
                            trail ? &job : nullptr, q);
            hc ^= 1;
            const int slice = slice_of(n);
            if (!trail && slice >= 0) record(in, false, out, false, slice, q);
        }
        if (trail && single > 0) launch_record_job(g, RecJob{F[(start + sw) & 1], nullptr, slice_ptr(single - 1)}, q);
        for (int n = single; n + 1 < T; n += 2, ++sw) {
            const float* in = F[(start + sw) & 1];
            float* out = F[(start + sw + 1) & 1];
            const int s0 = slice_of(n), s1 = slice_of(n + 1);
            const bool want_mid = (s0 >= 0 || s1 >= 0) && g.vps > 0;
            launch_fwd2_step(g, fwd2, in, out, psi, hc, ec, eps, wave[n], wave[n + 1],
                             partials + (int64_t)n * pl.per_step, partials + (int64_t)(n + 1) * pl.per_step,
                             want_mid ? mid : nullptr, q);
            hc ^= 1;
            ec ^= 1;
            if (s0 >= 0) record(in, false, mid, true, s0, q);    // E^n from the input, H^{n+1/2} intermediate
            if (s1 >= 0) record(mid, true, out, false, s1, q);   // E^{n+1} intermediate, H^{n+3/2} from the output
        }
        launch_loss_final(partials, T, pl.per_step, loss, loss_series, q);
    };
    const int rc = run_sequence(call_key(pl, 0, cfg, {eps, fields, psi, store, ws, loss, loss_series}), s, enqueue,
                                what, allow_graph);
    if (rc) return rc;
    rec->problem_hash = pl.hash;
    rec->dtype = cfg->dtype;
    rec->k = cfg->k;
    rec->steps = T;
    rec->consumed = 0;
    return FDTD_OK;
}

}  // namespace

extern "C" {

int store_config(const fdtd_problem_t* prob, const fdtd_store_cfg_t* cfg, fdtd_store_info_t* info) {
    if (!info) return fail(FDTD_EINVAL, "info must not be NULL");
    Plan pl;
    int rc = make_plan(prob, cfg, &pl);
    if (rc) return rc;
    *info = pl.info;
    return FDTD_OK;
}

int fdtd_forward(const fdtd_problem_t* prob, const fdtd_store_cfg_t* cfg, const float* eps, float* fields,
                 float* psi, void* store, void* workspace, double* loss, double* loss_series,
                 fdtd_record_t* rec, void* stream) {
    Plan pl;
    int rc = make_plan(prob, cfg, &pl);
    if (rc) return rc;
    if (!eps || !fields || !psi || !store || !workspace || !loss || !rec)
        return fail(FDTD_EINVAL, "fdtd_forward: eps, fields, psi, store, workspace, loss and rec must not be NULL");
    return forward_with(pl, prob, cfg, eps, fields, psi, store, (char*)workspace, loss, loss_series, rec,
                        (hipStream_t)stream, true, "fdtd_forward");
}

int fdtd_forward_noalloc(const fdtd_problem_t* prob, const fdtd_store_cfg_t* cfg, const float* eps, float* fields,
                         float* psi, void* store, double* loss, double* loss_series, fdtd_record_t* rec,
                         void* stream) {
    Plan pl;
    int rc = make_plan(prob, cfg, &pl);
    if (rc) return rc;
    if (!eps || !fields || !psi || !store || !loss || !rec)
        return fail(FDTD_EINVAL, "fdtd_forward_noalloc: eps, fields, psi, store, loss and rec must not be NULL");
    const uint64_t need = pl.ws_fields + pl.info.fields_bytes;   // tables, partials, staging, one field buffer
    if (need > (uint64_t)FDTD_NOALLOC_SCRATCH_BYTES)
        return fail(FDTD_EINVAL, "fdtd_forward_noalloc: the problem needs %llu bytes of scratch, more than the %llu "
                    "the library holds (workspace_bytes - fields_bytes must not exceed FDTD_NOALLOC_SCRATCH_BYTES)",
                    (unsigned long long)need, (unsigned long long)FDTD_NOALLOC_SCRATCH_BYTES);
    char* ws = nullptr;
    rc = scratch_for_current_device(&ws);
    if (rc) return rc;
    // launched directly: graph capture and instantiation would allocate
    return forward_with(pl, prob, cfg, eps, fields, psi, store, ws, loss, loss_series, rec, (hipStream_t)stream,
                        false, "fdtd_forward_noalloc");
}

int fdtd_backward(const fdtd_problem_t* prob, const fdtd_store_cfg_t* cfg, const float* eps, float* fields,
                  const void* store, void* workspace, float* adj_fields, float* adj_psi,
                  const double* grad_scale, double* grad_eps, fdtd_record_t* rec, void* stream) {
    Plan pl;
    int rc = make_plan(prob, cfg, &pl);
    if (rc) return rc;
    if (!rec) return fail(FDTD_EINVAL, "fdtd_backward: rec must not be NULL");
    if (rec->problem_hash != pl.hash || rec->dtype != cfg->dtype || rec->k != cfg->k || rec->steps != prob->steps)
        return fail(FDTD_ESTORE, "fdtd_backward: the record belongs to a different problem or store config");
    if (rec->consumed)
        return fail(FDTD_ESTATE, "fdtd_backward: record already consumed (the fields were reversed)");
    if (!eps || !fields || !store || !workspace || !adj_fields || !adj_psi || !grad_eps)
        return fail(FDTD_EINVAL, "fdtd_backward: device pointers must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)workspace;
    Grid g = pl.g;
    g.coef = (const float*)(ws + pl.ws_coef);
    g.src_profile = (const float*)(ws + pl.ws_profile);
    g.msrc_profile = (const float*)(ws + pl.ws_mprofile);

    const int T = prob->steps, k = cfg->k, ip = cfg->interp;
    const int64_t N = g.N;
    float* Fp[2] = {fields, (float*)(ws + pl.ws_fields)};                       // primal
    float* Fa[2] = {adj_fields, (float*)(ws + pl.ws_fields + pl.info.fields_bytes)};   // adjoint
    const float* wave = prob->src_wave;
    auto mwave = [&](int n) { return pl.msrc_volume > 0 ? prob->msrc_wave[n] : 0.0f; };
    Tiling adj = pl.adj;
    const bool two = pl.rev_steps == 2;
    float* mid = (float*)(ws + pl.ws_mid);
    float* stash = (float*)(ws + pl.ws_stash);
    std::vector<int32_t> order_adj, order_rev, order_rev2;
    tile_order(pl, 1, order_adj);
    adj.order = (const int32_t*)(ws + pl.ws_order_adj);
    Tiling rev = pl.rev, rev2 = pl.rev2;
    tile_order(pl, 3, order_rev);
    if (!order_rev.empty()) rev.order = (const int32_t*)(ws + pl.ws_order_rev);
    if (two) {
        tile_order(pl, 4, order_rev2);
        if (!order_rev2.empty()) rev2.order = (const int32_t*)(ws + pl.ws_order_rev2);
    }
    auto enqueue = [&](hipStream_t q) {
        put_tables(pl, prob, ws, q);
        launch_put(ws + pl.ws_order_adj, order_adj.data(), (long long)order_adj.size(), q);
        if (rev.order) launch_put(ws + pl.ws_order_rev, order_rev.data(), (long long)order_rev.size(), q);
        if (rev2.order) launch_put(ws + pl.ws_order_rev2, order_rev2.data(), (long long)order_rev2.size(), q);
        launch_fill(Fa[0], 6 * N, 0.0f, q);
        launch_fill(adj_psi, 2 * (long long)pl.psi_floats, 0.0f, q);
        launch_fill_f64(grad_eps, (long long)pl.info.design_cells, 0.0, q);
        Interp none;
        for (int t = 0; t < 4; ++t) { none.j[t] = -1; none.w[t] = 0.0f; }
        // the interface shell of the output state of reverse step n (E^n high faces,
        // H^{n-1/2} low faces), written before prim_rev of step n: E into its input
        // buffer FE (whose high-face E positions nothing else reads), H into its output
        // buffer FH
        // one step per sweep: the x-face shell cells go to row 0 of their plane (ShellJob.xrow),
        // where they fit when the face's rows fit in one row of the grid
        const int xrow = (!two && g.P >= 2 && g.my <= g.nx) ? 1 : 0;
        auto shell_for = [&](int n, float* FE, float* FH) {
            ShellJob j{FE, FH, store, interp_for(n, T, k, ip), n >= 1 ? interp_for(n - 1, T, k, ip) : none, 1,
                       n >= 1 ? 1 : 0};
            j.xrow = xrow;
            return j;
        };
        {
            ShellJob h{Fp[0], Fp[0], store, none, interp_for(T - 1, T, k, ip), 0, 1};   // H^{T-1/2}
            h.xrow = xrow;
            launch_inject_shell(g, h, q);
        }
        if (!two) {
            launch_inject_shell(g, shell_for(T - 1, Fp[0], Fp[1]), q);
            for (int n = T - 1; n >= 0; --n) {
                const int st = T - 1 - n;
                float* po = Fp[st & 1];
                float* pn = Fp[(st + 1) & 1];
                float* ao = Fa[st & 1];
                float* an = Fa[(st + 1) & 1];
                // the interior reversal reads the E part of the shell from po; the adjoint launch
                // then writes the shell of step n-1: E into pn (which the reversal has just
                // written: the input of step n-1), H into po (which it has finished reading)
                launch_prim_rev(g, rev, pl.box_o, pl.box_n, pl.rev_x0, xrow, po, pn, eps, ao, wave[n], mwave(n),
                                grad_eps, q);
                ShellJob next{};
                if (n >= 1) next = shell_for(n - 1, pn, po);
                launch_adj_step(g, adj, ao, an, eps, adj_psi, st & 1, n >= 1 ? &next : nullptr, q);
            }
        } else {
            // Two reverse steps per primal sweep: a single step first when T is odd, then the
            // pairs (m, m-1).  A pair needs step m's shell in mid (slice layout) and step m-1's
            // shell in its buffers (E into its input, H into its output); the adjoint launch of
            // the first step of the unit before writes the former, that of its second step the
            // latter.  Primal buffers alternate per sweep, adjoint buffers per step.
            auto mid_for = [&](int m) {
                ShellJob j = shell_for(m, mid, mid);
                j.slice = 1;
                return j;
            };
            int u = 0;                    // primal sweeps so far
            int n = T - 1;
            if (T & 1) {
                launch_inject_shell(g, shell_for(T - 1, Fp[0], Fp[1]), q);
                float* ao = Fa[0];
                float* an = Fa[1];
                launch_prim_rev(g, rev, pl.box_o, pl.box_n, pl.rev_x0, xrow, Fp[0], Fp[1], eps, ao, wave[n],
                                mwave(n), grad_eps, q);
                ShellJob next{};
                if (n >= 1) next = mid_for(n - 1);
                launch_adj_step(g, adj, ao, an, eps, adj_psi, 0, n >= 1 ? &next : nullptr, q);
                if (n >= 2) launch_inject_shell(g, shell_for(n - 2, Fp[1], Fp[0]), q);
                u = 1;
                n -= 1;
            } else {
                launch_inject_shell(g, mid_for(T - 1), q);
                launch_inject_shell(g, shell_for(T - 2, Fp[0], Fp[1]), q);
            }
            for (; n >= 1; n -= 2, ++u) {
                float* po = Fp[u & 1];
                float* pn = Fp[(u + 1) & 1];
                const int st = T - 1 - n;
                float* a0 = Fa[st & 1];
                float* a1 = Fa[(st + 1) & 1];
                launch_rev2(g, rev2, po, pn, eps, a0, wave[n], wave[n - 1], grad_eps, stash, mid, q);
                // the next pair (n-2, n-3): step n-2's shell into mid, step n-3's into pn (its
                // input: E) and po (its output: H)
                ShellJob ja{}, jb{};
                if (n >= 3) { ja = mid_for(n - 2); jb = shell_for(n - 3, pn, po); }
                launch_adj_step(g, adj, a0, a1, eps, adj_psi, st & 1, n >= 3 ? &ja : nullptr, q);
                launch_rev_pending(g, a1, grad_eps, stash, q);
                launch_adj_step(g, adj, a1, a0, eps, adj_psi, (st + 1) & 1, n >= 3 ? &jb : nullptr, q);
            }
        }
        if (grad_scale) launch_scale_grad(grad_eps, (long long)pl.info.design_cells, grad_scale, q);
    };
    rc = run_sequence(call_key(pl, 1, cfg, {eps, fields, store, workspace, adj_fields, adj_psi, grad_scale, grad_eps}),
                      s, enqueue, "fdtd_backward");
    if (rc) return rc;
    rec->consumed = 1;
    return FDTD_OK;
}

int fdtd_codec_roundtrip(int32_t dtype, const float* values, int64_t n_blocks, int64_t block_len, void* codes,
                         float* scales, float* decoded, void* stream) {
    if (dtype < FDTD_STORE_FP32 || dtype > FDTD_STORE_FP8_E4M3FN)
        return fail(FDTD_ESTORE, "unknown storage type %d", dtype);
    if (n_blocks < 0 || block_len < 0 || n_blocks > 0x7fffffff)
        return fail(FDTD_EINVAL, "fdtd_codec_roundtrip: bad block count or length");
    if (n_blocks == 0 || block_len == 0) return FDTD_OK;
    if (!values || !codes || !decoded || (dtype == FDTD_STORE_FP8_E4M3_SCALED && !scales))
        return fail(FDTD_EINVAL, "fdtd_codec_roundtrip: NULL buffer");
    launch_codec_roundtrip(dtype, values, n_blocks, block_len, codes, scales, decoded, (hipStream_t)stream);
    return check_hip("fdtd_codec_roundtrip");
}

int fdtd_set_graphs(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_graphs.mu);
    g_graphs.enabled = enable != 0;
    return FDTD_OK;
}

int fdtd_timing_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.enabled = enable != 0;
    g_timing.used = 0;
    return FDTD_OK;
}

int fdtd_timing_read(fdtd_kernel_time_t* out, int32_t max_kinds) {
    if (!out || max_kinds < 0) return fail(FDTD_EINVAL, "fdtd_timing_read: bad output buffer");
    std::lock_guard<std::mutex> lk(g_timing.mu);
    double total[K_NUM_KINDS] = {0};
    uint64_t count[K_NUM_KINDS] = {0};
    for (size_t t = 0; t < g_timing.used; ++t) {
        if (hipEventSynchronize(g_timing.pool[2 * t + 1]) != hipSuccess)
            return fail(FDTD_EHIP, "fdtd_timing_read: event synchronisation failed");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, g_timing.pool[2 * t], g_timing.pool[2 * t + 1]) != hipSuccess)
            return fail(FDTD_EHIP, "fdtd_timing_read: elapsed time unavailable");
        total[g_timing.kinds[t]] += ms;
        count[g_timing.kinds[t]] += 1;
    }
    int filled = 0;
    for (int kd = 0; kd < K_NUM_KINDS && filled < max_kinds; ++kd) {
        if (!count[kd]) continue;
        std::memset(&out[filled], 0, sizeof out[filled]);
        std::snprintf(out[filled].name, sizeof out[filled].name, "%s", kKindNames[kd]);
        out[filled].launches = count[kd];
        out[filled].total_ms = total[kd];
        ++filled;
    }
    return filled;
}

const char* fdtd_strerror(int code) {
    switch (code) {
        case FDTD_OK: return "ok";
        case FDTD_EINVAL: return "invalid argument";
        case FDTD_ECFL: return "Courant number outside (0, 1]";
        case FDTD_EREGION: return "box outside the interior";
        case FDTD_ESTORE: return "invalid store configuration or mismatched record";
        case FDTD_ESTATE: return "record already consumed";
        case FDTD_EHIP: return "HIP runtime error";
        case FDTD_ENONFINITE: return "non-finite loss";
        default: return "unknown error";
    }
}

const char* fdtd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
