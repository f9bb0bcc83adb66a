// Two forward Yee steps per sweep (temporal blocking of the forward time loop, gfx950).
//
// One sweep advances (E^n, H^{n-1/2}) in F0 to (E^{n+2}, H^{n+3/2}) in F1, so the fields
// and the PML auxiliaries cross HBM once for two steps instead of once per step.  The
// arithmetic of each half step is the one of the single-step sweep (forward.hip):
//   H^{m+1/2} = H^{m-1/2} - dt curl E^m          (forward differences)
//   E^{m+1}   = E^m + (dt / eps)(curl H^{m+1/2} - J^m)   (backward differences)
// with the CPML recursions inside the slabs, evaluated twice.
//
// Geometry.  A block owns W2 = 60 columns by HY = 12 rows of the grid and CZ planes.  Its
// threads (64 x (HY + 4), one wavefront per row) cover the owned tile plus two cells on
// each side in x and y.  Each half step shrinks the region that holds valid values by
// one cell on the side its differences look at:
//   E^n         lanes 0..63, rows 0..HY+3       (read from memory)
//   H^{n+1/2}   lanes 0..62, rows 0..HY+2       (needs E^n at +x, +y)
//   E^{n+1}     lanes 1..62, rows 1..HY+2       (needs H^{n+1/2} at -x, -y)
//   H^{n+3/2}   lanes 1..61, rows 1..HY+1
//   E^{n+2}     lanes 2..61, rows 2..HY+1       (the owned tile)
// Values outside a region are computed from whatever their neighbours hold and never
// used.  Along z the second step trails the first by one plane: iteration k evaluates
// H^{n+1/2}(k) and E^{n+1}(k), then H^{n+3/2}(k-1) and E^{n+2}(k-1), so a block marches
// from plane k0-2 to k0+CZ and stores planes k0..k0+CZ-1.
//
// LDS holds one plane of each of the four fields (E^n(k), H^{n+1/2}(k), E^{n+1}(k-1),
// H^{n+3/2}(k-1)) and two barriers per iteration order their writes and reads:
//   H1(k) -> sH1 | A | E1(k), H2(k-1) (reads sE1 = E1(k-1)); H2 -> sH2, E^n(k+1) -> sEn
//   | B | E2(k-1); E1(k) -> sE1.
//
// The H-side and E-side PML auxiliaries both ping-pong between the two copies of the
// PML buffer (a block reads the first step's inputs of its halo cells, which their
// owners update in the same launch).  With a recorder slice due on either step, the
// owners of the interface faces also write the intermediate values the recorder needs
// (H^{n+1/2} on the low faces, E^{n+1} on the high ones) into an FP32 buffer laid out
// as one kept step of the store.
#include "march.h"

namespace fdtd {

// CPML coefficients over the extended tile: x positions a-2 .. a+61, y positions
// j0-2 .. j0+HY+1, z positions k0-2 .. k0+CZ: [side 0 E / 1 H][b | a | kinv][position].
template <int HY, int CZ>
struct CoefTile2 {
    float x[2][3][TX];
    float y[2][3][HY + 4];
    float z[2][3][CZ + 3];
};

template <int HY, int CZ>
__device__ inline void fill_coef_tile2(const Grid& g, CoefTile2<HY, CZ>& ct, int a, int j0, int k0, int tid,
                                       int nthreads) {
    constexpr int NX = 6 * TX, NY = 6 * (HY + 4), NZ = 6 * (CZ + 3);
    for (int e = tid; e < NX + NY + NZ; e += nthreads) {
        if (e < NX) {
            const int side = e / (3 * TX), kind = (e / TX) % 3, pos = e % TX;
            ct.x[side][kind][pos] = coef_at(g, side, kind, a - 2 + pos, g.nx);
        } else if (e < NX + NY) {
            const int r = e - NX, side = r / (3 * (HY + 4)), kind = (r / (HY + 4)) % 3, pos = r % (HY + 4);
            ct.y[side][kind][pos] = coef_at(g, side, kind, j0 - 2 + pos, g.ny);
        } else {
            const int r = e - NX - NY, side = r / (3 * (CZ + 3)), kind = (r / (CZ + 3)) % 3, pos = r % (CZ + 3);
            ct.z[side][kind][pos] = coef_at(g, side, kind, k0 - 2 + pos, g.nz);
        }
    }
}

// Buffer resources and byte offsets of the PML copies of one two-step sweep.
struct Fwd2Bufs {
    rsrc_t F0, F1, psi, eps, src;
    uint32_t hin, hout, ein, eout;
};

// Loop-invariant per-lane offsets: the column (loads; OOB outside the grid), the owned
// cell (stores), the source box column, PML auxiliaries for loads and for stores.
struct Fwd2Lanes {
    uint32_t f, o, src;
    PsiLane pl, ps;
    bool ysl;                 // the row lies in a y slab (uniform across a wave)
};

// Inputs of iteration k, loaded one iteration ahead: E^n(k+1), H^{n-1/2}(k), eps(k),
// the source profile at k, and the PML auxiliaries of plane k (both sides).
struct In2 {
    float e1[3], h0[3], ep, sp;
    float ph[6], pe[6];
};

// State carried from iteration k-1 to k (all of the thread's own column; E^n(k) and
// E^{n+1}(k-1) of the own cell are read back from their LDS planes).
struct Carry2 {
    float h1[3];              // H^{n+1/2}(k-1)
    float h2x, h2y;           // H^{n+3/2}(k-2), the components a z difference takes
    float ep, sp;             // eps(k-1), source profile at k-1
    float ph1[6], pe1[6];     // PML auxiliaries after the first step at k-1
};

template <int SL>
__device__ __forceinline__ void load_in2(const Grid& g, const Fwd2Bufs& b, const Fwd2Lanes& L, bool live, int plane,
                                         uint32_t nb, int k, In2& d) {
    const int zk = bound(k, g.nz, g.periodic), z1 = bound(k + 1, g.nz, g.periodic);
    const uint32_t s1 = uni(z1 < 0 ? 0u : (uint32_t)(z1 * plane) << 2);
    bld3v(b.F0, z1 < 0 ? OOB : L.f, s1, nb, d.e1);
    const uint32_t sk = uni(zk < 0 ? 0u : (uint32_t)(zk * plane) << 2);
    const uint32_t vk = zk < 0 ? OOB : L.f;
    bld3v(b.F0, vk, sk + 3 * nb, nb, d.h0);
    const float ep = bldv(b.eps, vk, sk);
    d.ep = (live && zk >= 0) ? ep : 1.0f;
    uint32_t ss = 0;
    const bool sin = zk >= 0 && zk >= g.src_lo[2] && zk < g.src_hi[2];
    if (sin) ss = (uint32_t)((zk - g.src_lo[2]) * (g.src_hi[0] - g.src_lo[0]) * (g.src_hi[1] - g.src_lo[1])) << 2;
    d.sp = bldv(b.src, sin ? L.src : OOB, uni(ss));
    PsiPlane pH = psi_plane(g, 0, zk < 0 ? 0 : zk, b.hin), pE = psi_plane(g, 1, zk < 0 ? 0 : zk, b.ein);
    pH.zs = pE.zs = pH.zs && zk >= 0;
    PsiLane l = L.pl;
    if (zk < 0) l.x = l.y = l.z = OOB;
    bld_psi_s<SL>(b.psi, l, pH, d.ph);
    bld_psi_s<SL>(b.psi, l, pE, d.pe);
}

// Recorder values of an intermediate step at an owned cell: H^{n+1/2} on the low faces,
// E^{n+1} on the high faces, each face over its interior extent (the layout of one kept
// step of the store: blocks 2f and 2f+1 of face f).
__device__ __forceinline__ void mid_put(const Grid& g, float* mid, int x, int y, int z, const float h[3],
                                        const float e[3]) {
    const int P = g.P;
    const bool ix = x >= P && x < g.nx - P, iy = y >= P && y < g.ny - P, iz = z >= P && z < g.nz - P;
    if (x == P - 1 && iy && iz) {
        const long long u = (y - P) + (long long)g.my * (z - P);
        mid[block_offset(g, 0) + u] = h[1];
        mid[block_offset(g, 1) + u] = h[2];
    }
    if (y == P - 1 && ix && iz) {
        const long long u = (x - P) + (long long)g.mx * (z - P);
        mid[block_offset(g, 2) + u] = h[2];
        mid[block_offset(g, 3) + u] = h[0];
    }
    if (z == P - 1 && ix && iy) {
        const long long u = (x - P) + (long long)g.mx * (y - P);
        mid[block_offset(g, 4) + u] = h[0];
        mid[block_offset(g, 5) + u] = h[1];
    }
    if (x == g.nx - P && iy && iz) {
        const long long u = (y - P) + (long long)g.my * (z - P);
        mid[block_offset(g, 6) + u] = e[1];
        mid[block_offset(g, 7) + u] = e[2];
    }
    if (y == g.ny - P && ix && iz) {
        const long long u = (x - P) + (long long)g.mx * (z - P);
        mid[block_offset(g, 8) + u] = e[2];
        mid[block_offset(g, 9) + u] = e[0];
    }
    if (z == g.nz - P && ix && iy) {
        const long long u = (x - P) + (long long)g.mx * (y - P);
        mid[block_offset(g, 10) + u] = e[0];
        mid[block_offset(g, 11) + u] = e[1];
    }
}

// Per-thread constants of a two-step sweep.
struct Ctx2 {
    int lane, row, x, y, plane, k0, k1;
    bool live, own;
    uint32_t nb;
};

template <int HY>
using Plane2 = float[3][HY + 6][TX + 2];   // one LDS plane, padded by one cell on every side

// Iteration k of the two-step march (see the file header for the order of its phases).
template <int HY, int CZ, int SL>
__device__ __forceinline__ void iter2(const Grid& g, const Fwd2Bufs& b, const Fwd2Lanes& L, const Ctx2& c,
                                      Plane2<HY>& sEn, Plane2<HY>& sH1, Plane2<HY>& sE1, Plane2<HY>& sH2,
                                      const CoefTile2<HY, CZ>& ct, int k, const In2& in, Carry2& cr, float w0,
                                      float w1, float* mid, double& l0, double& l1) {
    const int lane = c.lane, row = c.row, lx = lane + 1, ly = row + 1;
    const int lz = k - (c.k0 - 2), lzp = lz > 0 ? lz - 1 : 0;
    const int zk = bound(k, g.nz, g.periodic), zp = bound(k - 1, g.nz, g.periodic);
    const bool cl = c.live && zk >= 0, clp = c.live && zp >= 0;
    const bool st1 = k >= c.k0 && k < c.k1;              // plane k is one of the block's own
    const bool st2 = k - 1 >= c.k0 && k - 1 < c.k1;      // plane k-1 is one of the block's own
    const float dt = g.dt;
    const uint32_t nb = c.nb;
    // ---- H^{n+1/2}(k) ----
    float h1[3], ph[6];
    #pragma unroll
    for (int t = 0; t < 6; ++t) ph[t] = in.ph[t];
    {
        float t[6];
        const float ex = sEn[0][ly][lx], ey = sEn[1][ly][lx], ez = sEn[2][ly][lx];   // E^n(k), own cell
        t[0] = sEn[2][ly + 1][lx] - ez;
        t[1] = in.e1[1] - ey;
        t[2] = in.e1[0] - ex;
        t[3] = sEn[2][ly][lx + 1] - ez;
        t[4] = sEn[1][ly][lx + 1] - ey;
        t[5] = sEn[0][ly + 1][lx] - ex;
        const PsiPlane pz = psi_plane(g, 0, zk < 0 ? 0 : zk, 0);
        if constexpr ((SL & 1) != 0) cpml_x(Cf{ct.x[1][0][lane], ct.x[1][1][lane], ct.x[1][2][lane]}, t, ph);
        if constexpr ((SL & 2) != 0) { if (L.ysl) cpml_y(Cf{ct.y[1][0][row], ct.y[1][1][row], ct.y[1][2][row]}, t, ph); }
        if constexpr ((SL & 4) != 0) { if (pz.zs && zk >= 0) cpml_z(Cf{ct.z[1][0][lz], ct.z[1][1][lz], ct.z[1][2][lz]}, t, ph); }
        h1[0] = cl ? in.h0[0] - dt * (t[0] - t[1]) : 0.0f;
        h1[1] = cl ? in.h0[1] - dt * (t[2] - t[3]) : 0.0f;
        h1[2] = cl ? in.h0[2] - dt * (t[4] - t[5]) : 0.0f;
    }
    sH1[0][ly][lx] = h1[0];
    sH1[1][ly][lx] = h1[1];
    sH1[2][ly][lx] = h1[2];
    __syncthreads();   // A
    // ---- E^{n+1}(k) ----
    float e1[3], pe[6];
    #pragma unroll
    for (int t = 0; t < 6; ++t) pe[t] = in.pe[t];
    {
        float t[6];
        t[0] = h1[2] - sH1[2][ly - 1][lx];
        t[1] = h1[1] - cr.h1[1];
        t[2] = h1[0] - cr.h1[0];
        t[3] = h1[2] - sH1[2][ly][lx - 1];
        t[4] = h1[1] - sH1[1][ly][lx - 1];
        t[5] = h1[0] - sH1[0][ly - 1][lx];
        const PsiPlane pz = psi_plane(g, 1, zk < 0 ? 0 : zk, 0);
        if constexpr ((SL & 1) != 0) cpml_x(Cf{ct.x[0][0][lane], ct.x[0][1][lane], ct.x[0][2][lane]}, t, pe);
        if constexpr ((SL & 2) != 0) { if (L.ysl) cpml_y(Cf{ct.y[0][0][row], ct.y[0][1][row], ct.y[0][2][row]}, t, pe); }
        if constexpr ((SL & 4) != 0) { if (pz.zs && zk >= 0) cpml_z(Cf{ct.z[0][0][lz], ct.z[0][1][lz], ct.z[0][2][lz]}, t, pe); }
        float u[3] = {t[0] - t[1], t[2] - t[3], t[4] - t[5]};
        const float jv = w0 * in.sp;   // 0 outside the source box
        u[0] -= g.src_comp == 0 ? jv : 0.0f;
        u[1] -= g.src_comp == 1 ? jv : 0.0f;
        u[2] -= g.src_comp == 2 ? jv : 0.0f;
        const float cc = dt_over_eps(dt, in.ep);
        e1[0] = cl ? sEn[0][ly][lx] + cc * u[0] : 0.0f;
        e1[1] = cl ? sEn[1][ly][lx] + cc * u[1] : 0.0f;
        e1[2] = cl ? sEn[2][ly][lx] + cc * u[2] : 0.0f;
    }
    if (c.own && st1) {
        if (in_box(c.x, c.y, k, g.det_lo, g.det_hi)) l0 += loss_term(g.loss, e1, h1);
        if (mid) mid_put(g, mid, c.x, c.y, k, h1, e1);
    }
    // ---- H^{n+3/2}(k-1) ----
    float h2[3], ph2[6];
    #pragma unroll
    for (int t = 0; t < 6; ++t) ph2[t] = cr.ph1[t];
    {
        float t[6];
        const float ex = sE1[0][ly][lx], ey = sE1[1][ly][lx], ez = sE1[2][ly][lx];   // E^{n+1}(k-1), own cell
        t[0] = sE1[2][ly + 1][lx] - ez;
        t[1] = e1[1] - ey;
        t[2] = e1[0] - ex;
        t[3] = sE1[2][ly][lx + 1] - ez;
        t[4] = sE1[1][ly][lx + 1] - ey;
        t[5] = sE1[0][ly + 1][lx] - ex;
        const PsiPlane pz = psi_plane(g, 0, zp < 0 ? 0 : zp, 0);
        if constexpr ((SL & 1) != 0) cpml_x(Cf{ct.x[1][0][lane], ct.x[1][1][lane], ct.x[1][2][lane]}, t, ph2);
        if constexpr ((SL & 2) != 0) { if (L.ysl) cpml_y(Cf{ct.y[1][0][row], ct.y[1][1][row], ct.y[1][2][row]}, t, ph2); }
        if constexpr ((SL & 4) != 0) { if (pz.zs && zp >= 0) cpml_z(Cf{ct.z[1][0][lzp], ct.z[1][1][lzp], ct.z[1][2][lzp]}, t, ph2); }
        h2[0] = clp ? cr.h1[0] - dt * (t[0] - t[1]) : 0.0f;
        h2[1] = clp ? cr.h1[1] - dt * (t[2] - t[3]) : 0.0f;
        h2[2] = clp ? cr.h1[2] - dt * (t[4] - t[5]) : 0.0f;
    }
    const uint32_t sp2 = uni(zp < 0 ? 0u : (uint32_t)(zp * c.plane) << 2);
    const uint32_t o2 = st2 ? L.o : OOB;
    bst3v(b.F1, o2, sp2 + 3 * nb, nb, h2);
    {
        PsiLane ls = L.ps;
        if (!st2) ls.x = ls.y = ls.z = OOB;
        PsiPlane pH = psi_plane(g, 0, zp < 0 ? 0 : zp, b.hout);
        pH.zs = pH.zs && zp >= 0;
        bst_psi_s<SL>(b.psi, ls, pH, ph2);
    }
    sH2[0][ly][lx] = h2[0];
    sH2[1][ly][lx] = h2[1];
    sH2[2][ly][lx] = h2[2];
    sEn[0][ly][lx] = in.e1[0];
    sEn[1][ly][lx] = in.e1[1];
    sEn[2][ly][lx] = in.e1[2];
    __syncthreads();   // B
    // ---- E^{n+2}(k-1) ----
    {
        float t[6], pe2[6];
        #pragma unroll
        for (int q = 0; q < 6; ++q) pe2[q] = cr.pe1[q];
        t[0] = h2[2] - sH2[2][ly - 1][lx];
        t[1] = h2[1] - cr.h2y;
        t[2] = h2[0] - cr.h2x;
        t[3] = h2[2] - sH2[2][ly][lx - 1];
        t[4] = h2[1] - sH2[1][ly][lx - 1];
        t[5] = h2[0] - sH2[0][ly - 1][lx];
        const PsiPlane pz = psi_plane(g, 1, zp < 0 ? 0 : zp, 0);
        if constexpr ((SL & 1) != 0) cpml_x(Cf{ct.x[0][0][lane], ct.x[0][1][lane], ct.x[0][2][lane]}, t, pe2);
        if constexpr ((SL & 2) != 0) { if (L.ysl) cpml_y(Cf{ct.y[0][0][row], ct.y[0][1][row], ct.y[0][2][row]}, t, pe2); }
        if constexpr ((SL & 4) != 0) { if (pz.zs && zp >= 0) cpml_z(Cf{ct.z[0][0][lzp], ct.z[0][1][lzp], ct.z[0][2][lzp]}, t, pe2); }
        float u[3] = {t[0] - t[1], t[2] - t[3], t[4] - t[5]};
        const float jv = w1 * cr.sp;
        u[0] -= g.src_comp == 0 ? jv : 0.0f;
        u[1] -= g.src_comp == 1 ? jv : 0.0f;
        u[2] -= g.src_comp == 2 ? jv : 0.0f;
        const float cc = dt_over_eps(dt, cr.ep);
        float e2[3];
        e2[0] = clp ? sE1[0][ly][lx] + cc * u[0] : 0.0f;   // E^{n+1}(k-1): sE1 still holds it
        e2[1] = clp ? sE1[1][ly][lx] + cc * u[1] : 0.0f;
        e2[2] = clp ? sE1[2][ly][lx] + cc * u[2] : 0.0f;
        bst3v(b.F1, o2, sp2, nb, e2);
        PsiLane ls = L.ps;
        if (!st2) ls.x = ls.y = ls.z = OOB;
        PsiPlane pE = psi_plane(g, 1, zp < 0 ? 0 : zp, b.eout);
        pE.zs = pE.zs && zp >= 0;
        bst_psi_s<SL>(b.psi, ls, pE, pe2);
        if (c.own && st2 && in_box(c.x, c.y, k - 1, g.det_lo, g.det_hi)) l1 += loss_term(g.loss, e2, h2);
    }
    sE1[0][ly][lx] = e1[0];
    sE1[1][ly][lx] = e1[1];
    sE1[2][ly][lx] = e1[2];
    // ---- carry to iteration k+1 ----
    #pragma unroll
    for (int q = 0; q < 3; ++q) cr.h1[q] = h1[q];
    cr.h2x = h2[0];
    cr.h2y = h2[1];
    cr.ep = in.ep;
    cr.sp = in.sp;
    #pragma unroll
    for (int t = 0; t < 6; ++t) { cr.ph1[t] = ph[t]; cr.pe1[t] = pe[t]; }
}

// The march of one tile of class SL: the prologue (E^n(k0-2) into LDS and registers,
// zero carries, the inputs of the first iteration), then iterations k0-2 .. k1, two per
// loop trip so that the inputs of iteration k+1 are loaded into the other register set
// before iteration k runs.
template <int HY, int CZ, int SL>
__device__ __forceinline__ void fwd2_tile(const Grid& g, const Fwd2Bufs& b, const Fwd2Lanes& L, const Ctx2& c,
                                          Plane2<HY>& sEn, Plane2<HY>& sH1, Plane2<HY>& sE1, Plane2<HY>& sH2,
                                          const CoefTile2<HY, CZ>& ct, float w0, float w1, float* mid, double& l0,
                                          double& l1) {
    Carry2 cr;
    float en[3];
    {
        const int zm = bound(c.k0 - 2, g.nz, g.periodic);
        const uint32_t sm = uni(zm < 0 ? 0u : (uint32_t)(zm * c.plane) << 2);
        bld3v(b.F0, zm < 0 ? OOB : L.f, sm, c.nb, en);
    }
    #pragma unroll
    for (int q = 0; q < 3; ++q) cr.h1[q] = 0.0f;
    cr.h2x = cr.h2y = 0.0f;
    cr.ep = 1.0f;
    cr.sp = 0.0f;
    #pragma unroll
    for (int t = 0; t < 6; ++t) { cr.ph1[t] = 0.0f; cr.pe1[t] = 0.0f; }
    In2 pin[2];
    load_in2<SL>(g, b, L, c.live, c.plane, c.nb, c.k0 - 2, pin[0]);
    #pragma unroll
    for (int q = 0; q < 3; ++q) {
        sEn[q][c.row + 1][c.lane + 1] = en[q];
        sE1[q][c.row + 1][c.lane + 1] = 0.0f;
    }
    __syncthreads();   // also publishes the coefficient tile
    const int cnt = c.k1 - c.k0 + 3;
    #pragma unroll 1
    for (int it = 0; it < cnt; it += 2) {
        const int k = c.k0 - 2 + it;
        if (it + 1 < cnt) load_in2<SL>(g, b, L, c.live, c.plane, c.nb, k + 1, pin[1]);
        iter2<HY, CZ, SL>(g, b, L, c, sEn, sH1, sE1, sH2, ct, k, pin[0], cr, w0, w1, mid, l0, l1);
        if (it + 1 < cnt) {
            if (it + 2 < cnt) load_in2<SL>(g, b, L, c.live, c.plane, c.nb, k + 2, pin[0]);
            iter2<HY, CZ, SL>(g, b, L, c, sEn, sH1, sE1, sH2, ct, k + 1, pin[1], cr, w0, w1, mid, l0, l1);
        }
    }
}

// Steps n and n+1: (E^n, H^{n-1/2}) in F0 -> (E^{n+2}, H^{n+3/2}) in F1.  PML copies:
// H side hcopy -> 1 - hcopy, E side ecopy -> 1 - ecopy.  w0, w1: source waveform at n and
// n + 1.  p0, p1: the detector partials of the two steps (one per tile meeting the
// detector).  mid: NULL, or the recorder buffer of the intermediate values.
template <int HY, int CZ>
__global__ __launch_bounds__(TX * (HY + 4)) void k_fwd2_step(Grid g, Tiling tl, const float* __restrict__ F0,
                                                             float* __restrict__ F1, float* __restrict__ psi,
                                                             int hcopy, int ecopy, const float* __restrict__ eps,
                                                             float w0, float w1, double* __restrict__ p0,
                                                             double* __restrict__ p1, float* __restrict__ mid) {
    __shared__ Plane2<HY> sEn, sH1, sE1, sH2;
    __shared__ CoefTile2<HY, CZ> ct;
    __shared__ double red[2][HY + 4];
    const int Lt = logical_tile(tl);
    const int tix = Lt % tl.ntx, tiy = (Lt / tl.ntx) % tl.nty, tiz = Lt / (tl.ntx * tl.nty);
    const int a = tix * W2, j0 = tiy * HY;
    Ctx2 c;
    c.k0 = tiz * CZ;
    c.k1 = min(c.k0 + CZ, g.nz);
    c.lane = threadIdx.x;
    c.row = threadIdx.y;
    c.x = a - 2 + c.lane;
    c.y = j0 - 2 + c.row;
    c.plane = g.nx * g.ny;
    const int N = (int)g.N;
    c.nb = (uint32_t)N << 2;
    const Col col = make_col(g, c.x, c.y);
    c.live = col.xy >= 0;
    c.own = c.lane >= 2 && c.lane < TX - 2 && c.row >= 2 && c.row < HY + 2 && c.x < g.nx && c.y < g.ny;
    Fwd2Bufs b;
    const uint32_t fbytes = (uint32_t)(6 * N) * 4u, psib = (uint32_t)g.psi_total * 4u;
    b.F0 = make_rsrc(F0, fbytes);
    b.F1 = make_rsrc(F1, fbytes);
    b.psi = make_rsrc(psi, 2 * psib);
    b.hin = hcopy ? psib : 0u;
    b.hout = hcopy ? 0u : psib;
    b.ein = ecopy ? psib : 0u;
    b.eout = ecopy ? 0u : psib;
    b.eps = make_rsrc(eps, (uint32_t)(c.plane * g.nz) * 4u);
    const int sxn = g.src_hi[0] - g.src_lo[0], syn = g.src_hi[1] - g.src_lo[1];
    b.src = make_rsrc(g.src_profile, (uint32_t)(sxn * syn * (g.src_hi[2] - g.src_lo[2])) * 4u);
    Fwd2Lanes L;
    L.f = lane_off(c.live, col.xy);
    L.o = lane_off(c.live && c.own, col.xy);
    L.src = lane_off(c.live && col.x >= g.src_lo[0] && col.x < g.src_hi[0] && col.y >= g.src_lo[1] &&
                         col.y < g.src_hi[1],
                     (col.x - g.src_lo[0]) + sxn * (col.y - g.src_lo[1]));
    L.pl = psi_lane(g, col, c.live);
    L.ps = psi_lane(g, col, c.live && c.own);
    L.ysl = col.sy >= 0;
    const int tid = c.row * TX + c.lane;
    fill_coef_tile2<HY, CZ>(g, ct, a, j0, c.k0, tid, TX * (HY + 4));   // published by the prologue's barrier

    // the tile's class: the slabs reached by the cells whose auxiliaries it reads
    const int sl = slab_class(g, a - 2, a + TX - 3, j0 - 2, j0 + HY + 1, c.k0 - 2, c.k0 + CZ);
    double l0 = 0.0, l1 = 0.0;
    switch (sl) {
        case 0: fwd2_tile<HY, CZ, 0>(g, b, L, c, sEn, sH1, sE1, sH2, ct, w0, w1, mid, l0, l1); break;
        case 1: fwd2_tile<HY, CZ, 1>(g, b, L, c, sEn, sH1, sE1, sH2, ct, w0, w1, mid, l0, l1); break;
        case 2: fwd2_tile<HY, CZ, 2>(g, b, L, c, sEn, sH1, sE1, sH2, ct, w0, w1, mid, l0, l1); break;
        case 3: fwd2_tile<HY, CZ, 3>(g, b, L, c, sEn, sH1, sE1, sH2, ct, w0, w1, mid, l0, l1); break;
        case 4: fwd2_tile<HY, CZ, 4>(g, b, L, c, sEn, sH1, sE1, sH2, ct, w0, w1, mid, l0, l1); break;
        case 5: fwd2_tile<HY, CZ, 5>(g, b, L, c, sEn, sH1, sE1, sH2, ct, w0, w1, mid, l0, l1); break;
        case 6: fwd2_tile<HY, CZ, 6>(g, b, L, c, sEn, sH1, sE1, sH2, ct, w0, w1, mid, l0, l1); break;
        default: fwd2_tile<HY, CZ, 7>(g, b, L, c, sEn, sH1, sE1, sH2, ct, w0, w1, mid, l0, l1); break;
    }
    // detector partials of this tile (tiles meeting the detector only; uniform per block)
    const int dx = tix - tl.dtx0, dy = tiy - tl.dty0, dz = tiz - tl.dtz0;
    if (dx < 0 || dy < 0 || dz < 0 || dx >= tl.dntx || dy >= tl.dnty || dz >= tl.dntz) return;
    for (int off = 32; off > 0; off >>= 1) {
        l0 += __shfl_xor(l0, off, 64);
        l1 += __shfl_xor(l1, off, 64);
    }
    if (c.lane == 0) { red[0][c.row] = l0; red[1][c.row] = l1; }
    __syncthreads();
    if (tid == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < HY + 4; ++w) { s0 += red[0][w]; s1 += red[1][w]; }
        const long long i = dx + (long long)tl.dntx * (dy + (long long)tl.dnty * dz);
        p0[i] = s0;
        p1[i] = s1;
    }
}

template <int HY, int CZ>
static void launch_fwd2_t(const Grid& g, const Tiling& t, const float* F0, float* F1, float* psi, int hcopy,
                          int ecopy, const float* eps, float w0, float w1, double* p0, double* p1, float* mid,
                          hipStream_t s) {
    launch_kernel(K_FWD_STEP2, k_fwd2_step<HY, CZ>, dim3(t.count), dim3(TX, HY + 4), s, g, t, F0, F1, psi, hcopy,
                  ecopy, eps, w0, w1, p0, p1, mid);
}

void launch_fwd2_step(const Grid& g, const Tiling& t, const float* F0, float* F1, float* psi, int hcopy, int ecopy,
                      const float* eps, float w0, float w1, double* p0, double* p1, float* mid, hipStream_t s) {
    if (t.cz == 16) launch_fwd2_t<12, 16>(g, t, F0, F1, psi, hcopy, ecopy, eps, w0, w1, p0, p1, mid, s);
    else launch_fwd2_t<12, 8>(g, t, F0, F1, psi, hcopy, ecopy, eps, w0, w1, p0, p1, mid, s);
}

}  // namespace fdtd
