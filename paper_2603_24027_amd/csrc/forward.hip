// Forward Yee step with convolutional PML, interface recorder and detector loss (gfx950).
//
// One step n is one fused z-marching sweep (march.h):
//   H^{n+1/2} = H^{n-1/2} - dt curl E^n              (forward differences)
//   E^{n+1}   = E^n + (dt / eps)(curl H^{n+1/2} - J^n)  (backward differences)
// with the CPML recursions psi <- b psi + a g inside the slabs, on kept steps
// the interface shell (E^n on the high faces and H^{n+1/2} on the low faces;
// Section 2: the interface slices are recorded during the forward simulation)
// and the per-tile FP64 partial of sum_D |E^{n+1}|^2.
// The sweep's field and auxiliary stores carry device scope (cache-policy bit sc1):
// they write through the XCD's L2 rather than leaving dirty lines for the
// writeback at the end of every launch (measured: about 1 us of 38 per step at 128^3).
#ifndef FDTD_FWD_ST_AUX
#define FDTD_FWD_ST_AUX 16
#endif
#define FDTD_ST_AUX FDTD_FWD_ST_AUX
#include "march.h"

#include <algorithm>
#include <cstring>

namespace fdtd {

__global__ void k_fill(float* p, long long n, float v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_f64(double* p, long long n, double v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// Host values (32-bit words) written into device memory by kernel launches that carry
// them as arguments (PUT_CHUNK words per launch): no host staging buffer and no copy
// from pageable memory, and a captured graph holds the values themselves.
struct PutChunk {
    uint32_t v[PUT_CHUNK];
};

__global__ __launch_bounds__(256) void k_put(uint32_t* __restrict__ dst, int n, PutChunk c) {
    for (int i = threadIdx.x; i < n; i += 256) dst[i] = c.v[i];
}

void launch_put(void* dst, const void* host, long long n, hipStream_t s) {
    for (long long o = 0; o < n; o += PUT_CHUNK) {
        const int m = (int)std::min<long long>(PUT_CHUNK, n - o);
        PutChunk c;
        std::memcpy(c.v, (const uint32_t*)host + o, (size_t)m * sizeof(uint32_t));
        std::memset(c.v + m, 0, (size_t)(PUT_CHUNK - m) * sizeof(uint32_t));
        launch_kernel(K_PUT, k_put, dim3(1), dim3(256), s, (uint32_t*)dst + o, m, c);
    }
}

void launch_fill(float* p, long long n, float v, hipStream_t s) {
    if (n <= 0) return;
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    launch_kernel(K_FILL, k_fill, dim3((unsigned)blocks), dim3(256), s, p, n, v);
}

void launch_fill_f64(double* p, long long n, double v, hipStream_t s) {
    if (n <= 0) return;
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    launch_kernel(K_FILL, k_fill_f64, dim3((unsigned)blocks), dim3(256), s, p, n, v);
}

// The six curl-E differences of the H half at extended-plane position (ex, ey)
// from the LDS planes of E^n at z (cur) and z + 1 (nxt).
template <int TY>
__device__ inline void h_terms(const float (*cur)[TY + 2][EXT], const float (*nxt)[TY + 2][EXT], int ex, int ey,
                               float t[6]) {
    const float exc = cur[0][ey][ex], eyc = cur[1][ey][ex], ezc = cur[2][ey][ex];
    t[0] = cur[2][ey + 1][ex] - ezc;   // (Hx, y, +, Ez)
    t[1] = nxt[1][ey][ex] - eyc;       // (Hx, z, -, Ey)
    t[2] = nxt[0][ey][ex] - exc;       // (Hy, z, +, Ex)
    t[3] = cur[2][ey][ex + 1] - ezc;   // (Hy, x, -, Ez)
    t[4] = cur[1][ey][ex + 1] - eyc;   // (Hz, x, +, Ey)
    t[5] = cur[0][ey + 1][ex] - exc;   // (Hz, y, -, Ex)
}

// Buffer resources of one forward sweep.
struct FwdBufs {
    rsrc_t F0, F1, psi, eps, src, msrc;              // fields in / out (E then H), both PML copies
    uint32_t hin, hout;                              // byte offsets of the H-side PML copies in / out
};

// Loop-invariant per-lane byte offsets of the forward sweep (OOB where nothing is
// read or written): E^n of the own column (boundary rule, also for idle lanes, whose
// values serve as neighbours) and of the ring position; the own cell (live lanes);
// the halo cell; the source box column; PML auxiliaries of the own and halo cells.
struct FwdLanes {
    uint32_t eo, er, o, hc, src, m, mh;       // ... and the magnetic-current sheet (own, halo)
    PsiLane po, ph;
    bool ysl;                 // the own row lies in a y slab (uniform across a wave)
};

// Everything the forward sweep reads from memory for plane k of its column:
// E^n of plane k+1 (own cell and the LDS-ring position), H^{n-1/2} of plane k
// (own cell and the halo cell), eps, the source profile (0 outside the source box)
// and the PML auxiliaries of plane k (those of the axes the tile's class reaches).
struct PlaneIn {
    float e1[3], er[3], h0[3], hh0[3], ep, sp;
    float ph[6], pe[6], phh[6];
};

__device__ __forceinline__ uint32_t src_plane(const Grid& g, int k, uint32_t lane_src, uint32_t& s) {
    const bool in = k >= g.src_lo[2] && k < g.src_hi[2];
    s = uni(in ? (uint32_t)((k - g.src_lo[2]) * (g.src_hi[0] - g.src_lo[0]) * (g.src_hi[1] - g.src_lo[1])) << 2 : 0u);
    return in ? lane_src : OOB;
}

// Loads of plane k's inputs (out-of-domain and out-of-slab values read as 0).
template <int TY, int SL>
__device__ __forceinline__ void load_plane_in(const Grid& g, const FwdBufs& b, const FwdLanes& L,
                                              const FwdCtx<TY>& c, int k, PlaneIn& d) {
    const uint32_t nb = (uint32_t)c.N << 2;
    const int z1 = bound(k + 1, g.nz, g.periodic);
    const uint32_t s1 = uni(z1 < 0 ? 0u : (uint32_t)(z1 * c.plane) << 2);
    const uint32_t sk = uni((uint32_t)(k * c.plane) << 2);
    const PsiPlane pH = psi_plane(g, 0, k, b.hin), pE = psi_plane(g, 1, k, 0);
    // loads that only some waves use (rows 0-3 hold the LDS ring, rows 0-1 the halo cells),
    // issued first and only by those waves: the waits for the loads every wave issues
    // below then cover them too, so the counts stay exact
    #pragma unroll
    for (int q = 0; q < 3; ++q) { d.er[q] = 0.0f; d.hh0[q] = 0.0f; }
    #pragma unroll
    for (int q = 0; q < 6; ++q) d.phh[q] = 0.0f;
    if (c.row < 4) bld3v(b.F0, z1 < 0 ? OOB : L.er, s1, nb, d.er);
    if (c.row < 2) {
        bld3v(b.F0, L.hc, sk + 3 * nb, nb, d.hh0);
        bld_psi_s<SL>(b.psi, L.ph, pH, d.phh);
    }
    bld3v(b.F0, z1 < 0 ? OOB : L.eo, s1, nb, d.e1);
    bld3v(b.F0, L.o, sk + 3 * nb, nb, d.h0);
    const float ep = bldv(b.eps, L.o, sk);
    d.ep = c.live ? ep : 1.0f;
    uint32_t ss;
    const uint32_t vs = src_plane(g, k, L.src, ss);
    d.sp = bldv(b.src, vs, ss);
    bld_psi_s<SL>(b.psi, L.po, pH, d.ph);
    bld_psi_s<SL>(b.psi, L.po, pE, d.pe);
}

// One plane k of the forward sweep: publish E^n(k+1) to LDS, H^{n+1/2}(k) on the own
// and halo cells, then E^{n+1}(k) on the own cell.  `in` holds the plane's inputs,
// loaded one plane ahead.  All stores are unconditional buffer stores (dropped for
// idle lanes and cells outside a slab).  SL: the tile's class (slab_class).
template <int TY, int CZ, bool MS, int SL>
__device__ __forceinline__ void fwd_plane(const Grid& g, const FwdBufs& b, const FwdLanes& L, const FwdCtx<TY>& c,
                                          float (*sE)[3][TY + 2][EXT], float (*sH)[TY + 1][TX + 1],
                                          const CoefTile<TY, CZ>& ct, int lz, int cur, int k,
                                          const PlaneIn& in, float eo[3], float& hx_prev, float& hy_prev, double& e2,
                                          float wave, float mwave) {
    const int nxt = 1 - cur;
    const int x = c.x, y = c.y, row = c.row, lane = c.lane;
    const uint32_t nb = (uint32_t)c.N << 2;
    const uint32_t sk = uni((uint32_t)(k * c.plane) << 2);
    const PsiPlane pH = psi_plane(g, 0, k, b.hout), pE = psi_plane(g, 1, k, 0);
    float ph[6], phh[6], pe[6];
    #pragma unroll
    for (int t = 0; t < 6; ++t) { ph[t] = in.ph[t]; phh[t] = in.phh[t]; pe[t] = in.pe[t]; }
    // ---- E^n of plane k+1 into LDS ----
    #pragma unroll
    for (int q = 0; q < 3; ++q) sE[nxt][q][row + 1][lane + 1] = in.e1[q];
    if (c.rlx >= 0) {
        #pragma unroll
        for (int q = 0; q < 3; ++q) sE[nxt][q][c.rly][c.rlx] = in.er[q];
    }
    __syncthreads();
    // ---- first half: H^{n+1/2} on the own cell and the halo cell ----
    float mp = 0.0f, mph = 0.0f;
    if constexpr (MS) {
        // the magnetic-current sheet (a separate instantiation): only planes that carry it
        // load it, under a branch that is uniform per block and waits for its own loads
        uint32_t ms;
        if (box_plane(g.msrc_lo, g.msrc_hi, k, ms)) {
            mp = bldv(b.msrc, L.m, ms);
            mph = bldv(b.msrc, L.mh, ms);
        }
    }
    float h[3];
    {
        float t[6];
        h_terms<TY>(sE[cur], sE[nxt], lane + 1, row + 1, t);
        if constexpr ((SL & 1) != 0) cpml_x(cf_x(ct, 1, lane + 1), t, ph);
        if constexpr ((SL & 2) != 0) { if (L.ysl) cpml_y(cf_y(ct, 1, row + 1), t, ph); }
        if constexpr ((SL & 4) != 0) { if (pH.zs) cpml_z(cf_z(ct, 1, lz), t, ph); }
        const float dt = g.dt;
        const float m = MS ? dt * mwave * mp : 0.0f;     // magnetic current (0 outside its sheet)
        h[0] = c.live ? in.h0[0] - dt * (t[0] - t[1]) - (g.msrc_comp == 0 ? m : 0.0f) : 0.0f;
        h[1] = c.live ? in.h0[1] - dt * (t[2] - t[3]) - (g.msrc_comp == 1 ? m : 0.0f) : 0.0f;
        h[2] = c.live ? in.h0[2] - dt * (t[4] - t[5]) - (g.msrc_comp == 2 ? m : 0.0f) : 0.0f;
    }
    bst3v(b.F1, L.o, sk + 3 * nb, nb, h);
    bst_psi_s<SL>(b.psi, L.po, pH, ph);
    sH[0][row + 1][lane + 1] = h[0];
    sH[1][row + 1][lane + 1] = h[1];
    sH[2][row + 1][lane + 1] = h[2];
    if (c.hex >= 0) {
        float hh[3] = {0.0f, 0.0f, 0.0f};
        if (c.hc.xy >= 0) {
            float t[6];
            h_terms<TY>(sE[cur], sE[nxt], c.hex, c.hey, t);
            cpml_axes<SL>(cf_x(ct, 1, c.hex), cf_y(ct, 1, c.hey), cf_z(ct, 1, lz), t, phh);
            const float dt = g.dt;
            const float m = MS ? dt * mwave * mph : 0.0f;
            hh[0] = in.hh0[0] - dt * (t[0] - t[1]) - (g.msrc_comp == 0 ? m : 0.0f);
            hh[1] = in.hh0[1] - dt * (t[2] - t[3]) - (g.msrc_comp == 1 ? m : 0.0f);
            hh[2] = in.hh0[2] - dt * (t[4] - t[5]) - (g.msrc_comp == 2 ? m : 0.0f);
        }
        sH[0][c.hey][c.hex] = hh[0];
        sH[1][c.hey][c.hex] = hh[1];
        sH[2][c.hey][c.hex] = hh[2];
    }
    __syncthreads();
    // ---- second half: E^{n+1} on the own cell ----
    float t[6];
    t[0] = h[2] - sH[2][row][lane + 1];       // (Ex, y, +, Hz)
    t[1] = h[1] - hy_prev;                    // (Ex, z, -, Hy)
    t[2] = h[0] - hx_prev;                    // (Ey, z, +, Hx)
    t[3] = h[2] - sH[2][row + 1][lane];       // (Ey, x, -, Hz)
    t[4] = h[1] - sH[1][row + 1][lane];       // (Ez, x, +, Hy)
    t[5] = h[0] - sH[0][row][lane + 1];       // (Ez, y, -, Hx)
    if constexpr ((SL & 1) != 0) cpml_x(cf_x(ct, 0, lane + 1), t, pe);
    if constexpr ((SL & 2) != 0) { if (L.ysl) cpml_y(cf_y(ct, 0, row + 1), t, pe); }
    if constexpr ((SL & 4) != 0) { if (pE.zs) cpml_z(cf_z(ct, 0, lz), t, pe); }
    bst_psi_s<SL>(b.psi, L.po, pE, pe);
    float u[3] = {t[0] - t[1], t[2] - t[3], t[4] - t[5]};
    const float jv = wave * in.sp;   // 0 outside the source box
    u[0] -= g.src_comp == 0 ? jv : 0.0f;
    u[1] -= g.src_comp == 1 ? jv : 0.0f;
    u[2] -= g.src_comp == 2 ? jv : 0.0f;
    const float cc = dt_over_eps(g.dt, in.ep);
    float e[3];
    e[0] = eo[0] + cc * u[0];
    e[1] = eo[1] + cc * u[1];
    e[2] = eo[2] + cc * u[2];
    bst3v(b.F1, L.o, sk, nb, e);
    if (c.live && in_box(x, y, k, g.det_lo, g.det_hi)) e2 += loss_term(g.loss, e, h);
    hx_prev = h[0];
    hy_prev = h[1];
    eo[0] = in.e1[0]; eo[1] = in.e1[1]; eo[2] = in.e1[2];
}

// The z-march of one tile of class SL over planes [k0, k1): the prologue (E^n planes
// k0-1 and k0 into LDS, H^{n+1/2} of the own column at k0-1, the inputs of plane k0),
// then the planes, unrolled and software-pipelined: the loads of plane k+1 are issued
// before the stores of plane k into the other of two register sets, so no wait for
// them also waits for those stores (loads and stores retire in order).  Returns the
// tile's detector term of this thread.
template <int TY, int CZ, bool MS, int SL>
__device__ __forceinline__ double fwd_tile(const Grid& g, const FwdBufs& b, const FwdLanes& Ln, const FwdCtx<TY>& c,
                                           float (*sE)[3][TY + 2][EXT], float (*sH)[TY + 1][TX + 1],
                                           const CoefTile<TY, CZ>& ct, int k0, int k1, float wave, float mwave) {
    const int lane = c.lane, row = c.row, plane = c.plane;
    const uint32_t nb = (uint32_t)c.N << 2;
    PlaneIn pin[2];
    float eo[3];                       // E^n of the own cell on the current plane
    float hx_prev, hy_prev;            // H^{n+1/2} of the own cell on the previous plane
    {
        const int zm = bound(k0 - 1, g.nz, g.periodic);
        const uint32_t sm = uni(zm < 0 ? 0u : (uint32_t)(zm * plane) << 2), s0 = uni((uint32_t)(k0 * plane) << 2);
        float a[3], ra[3], rb[3], h0[3], p[6];
        bld3v(b.F0, zm < 0 ? OOB : Ln.eo, sm, nb, a);
        bld3v(b.F0, Ln.eo, s0, nb, eo);
        bld3v(b.F0, zm < 0 ? OOB : Ln.er, sm, nb, ra);
        bld3v(b.F0, Ln.er, s0, nb, rb);
        const bool pro = c.live && zm >= 0;
        bld3v(b.F0, zm < 0 ? OOB : Ln.o, sm + 3 * nb, nb, h0);
        PsiPlane pm = psi_plane(g, 0, zm < 0 ? 0 : zm, b.hin);
        pm.zs = pm.zs && zm >= 0;
        PsiLane lm = Ln.po;
        if (zm < 0) lm.x = lm.y = lm.z = OOB;
        bld_psi_s<SL>(b.psi, lm, pm, p);
        float mpm = 0.0f;
        if constexpr (MS) {
            uint32_t msm = 0;
            const bool mzm = zm >= 0 && box_plane(g.msrc_lo, g.msrc_hi, zm, msm);
            mpm = bldv(b.msrc, mzm ? Ln.m : OOB, msm);
        }
        load_plane_in<TY, SL>(g, b, Ln, c, k0, pin[0]);
        #pragma unroll
        for (int q = 0; q < 3; ++q) {
            sE[0][q][row + 1][lane + 1] = a[q];
            sE[1][q][row + 1][lane + 1] = eo[q];
        }
        if (c.rlx >= 0) {
            #pragma unroll
            for (int q = 0; q < 3; ++q) { sE[0][q][c.rly][c.rlx] = ra[q]; sE[1][q][c.rly][c.rlx] = rb[q]; }
        }
        __syncthreads();   // also publishes the coefficient tile
        float t[6];
        h_terms<TY>(sE[0], sE[1], lane + 1, row + 1, t);
        cpml_axes<SL>(cf_x(ct, 1, lane + 1), cf_y(ct, 1, row + 1), cf_z(ct, 1, 0), t, p);
        const float m = g.dt * mwave * mpm;
        hx_prev = pro ? h0[0] - g.dt * (t[0] - t[1]) - (g.msrc_comp == 0 ? m : 0.0f) : 0.0f;
        hy_prev = pro ? h0[1] - g.dt * (t[2] - t[3]) - (g.msrc_comp == 1 ? m : 0.0f) : 0.0f;
    }
    __syncthreads();   // the first plane overwrites sE[0], which the prologue has just read
    double e2 = 0.0;
    #pragma unroll
    for (int kk = 0; kk < CZ; ++kk) {
        const int k = k0 + kk;
        if (kk + 1 < CZ)   // inputs of the next plane (an unused valid plane past the end of the grid)
            load_plane_in<TY, SL>(g, b, Ln, c, min(k + 1, g.nz - 1), pin[(kk + 1) & 1]);
        if (k < k1)
            fwd_plane<TY, CZ, MS, SL>(g, b, Ln, c, sE, sH, ct, kk + 1, (kk + 1) & 1, k, pin[kk & 1], eo, hx_prev,
                                      hy_prev, e2, wave, mwave);
    }
    return e2;
}

// One full forward step n: (E^n, H^{n-1/2}) in F0 -> (E^{n+1}, H^{n+1/2}) in F1 (each E
// then H, 3 components of N cells).  The PML buffer holds two copies of the auxiliaries:
// the H-side ones ping-pong (copy hcopy -> 1 - hcopy), the E-side ones live in copy 0
// and are updated in place.  Each block runs the code of its tile's class: the PML
// auxiliaries of an axis are loaded, updated and stored only by tiles that one of that
// axis's slabs reaches (elsewhere they would all be out-of-range no-ops, and issuing
// them had cost a third of the sweep's time).
// With a magnetic-current sheet the sweep asks for 4 waves per SIMD: left free it
// takes more than 128 vector registers (3 waves, 24 % slower); held to 128 it spills
// only scalars, into vector-register lanes.
#ifndef FDTD_FWD_WAVES
#define FDTD_FWD_WAVES 1
#endif
// One face cell and side of a RecJob: both tangential components from the field
// buffer into the kept step, in its storage type.
template <int DT>
__device__ inline void rec_cell(const Grid& g, const RecJob& j, int t) {
    const int face = g.my * g.mz + g.mx * g.mz + g.mx * g.my;   // < 2^31: 24 N < 2^31
    if (t >= 2 * face) return;
    const bool high = t >= face;
    if (high) t -= face;
    void* dst = high ? j.dst_e : j.dst_h;
    if (!dst) return;
    const FaceCell f = face_cell(g, t, high);
    const long long N = g.N;
    const float* A = high ? j.F : j.F + 3 * N;                 // E on the high faces, H on the low ones
    const long long idx = f.x + (long long)g.nx * (f.y + (long long)g.ny * f.z);
    store_code<DT>(dst, block_offset(g, f.blk) + f.u, A[f.c0 * N + idx]);
    store_code<DT>(dst, block_offset(g, f.blk + 1) + f.u, A[f.c1 * N + idx]);
}

// the storage type is uniform over the launch: one branch per wave
__device__ inline void rec_cell_any(const Grid& g, const RecJob& j, int t) {
    switch (g.dtype) {
        case 0: rec_cell<0>(g, j, t); break;
        case 1: rec_cell<1>(g, j, t); break;
        case 2: rec_cell<2>(g, j, t); break;
        case 3: rec_cell<3>(g, j, t); break;
        case 4: rec_cell<4>(g, j, t); break;
        case 5: rec_cell<5>(g, j, t); break;
        case 6: rec_cell<6>(g, j, t); break;
        case 7: rec_cell<7>(g, j, t); break;
        case 8: rec_cell<8>(g, j, t); break;
        default: rec_cell<9>(g, j, t); break;
    }
}

__global__ __launch_bounds__(256) void k_record_job(Grid g, RecJob j) {
    rec_cell_any(g, j, (int)blockIdx.x * 256 + (int)threadIdx.x);
}

template <int TY, int CZ, bool MS>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(MS ? 4 : FDTD_FWD_WAVES))) void k_fwd_step(
    Grid g, Tiling tl, const float* __restrict__ F0, float* __restrict__ F1, float* __restrict__ psi, int hcopy,
    const float* __restrict__ eps, float wave, float mwave, double* __restrict__ partials, RecJob job) {
    __shared__ float sE[2][3][TY + 2][EXT];
    __shared__ float sH[3][TY + 1][TX + 1];
    __shared__ CoefTile<TY, CZ> ct;
    __shared__ double red[TY];
    if ((int)blockIdx.x >= tl.count) {   // trailing workgroups: interface values of kept steps
        rec_cell_any(g, job, ((int)blockIdx.x - tl.count) * (TX * TY) + (int)(threadIdx.y * TX + threadIdx.x));
        return;
    }
    const int L = logical_tile(tl);
    const int tix = L % tl.ntx, tiy = (L / tl.ntx) % tl.nty, tiz = L / (tl.ntx * tl.nty);
    FwdCtx<TY> c;
    c.i0 = tix * TX;
    c.j0 = tiy * TY;
    const int k0 = tiz * CZ;
    const int k1 = min(k0 + CZ, g.nz);
    c.lane = threadIdx.x;
    c.row = threadIdx.y;
    c.tid = c.row * TX + c.lane;
    c.x = c.i0 + c.lane;
    c.y = c.j0 + c.row;
    c.live = c.x < g.nx && c.y < g.ny;
    c.N = (int)g.N;
    c.P = g.P;
    c.plane = g.nx * g.ny;
    const int N = c.N, lane = c.lane, row = c.row;
    FwdBufs b;
    const uint32_t fbytes = (uint32_t)(6 * N) * 4u, psib = (uint32_t)g.psi_total * 4u;
    b.F0 = make_rsrc(F0, fbytes);
    b.F1 = make_rsrc(F1, fbytes);
    b.psi = make_rsrc(psi, 2 * psib);
    b.hin = hcopy ? psib : 0u;
    b.hout = hcopy ? 0u : psib;
    b.eps = make_rsrc(eps, (uint32_t)(c.plane * g.nz) * 4u);
    const int sxn = g.src_hi[0] - g.src_lo[0], syn = g.src_hi[1] - g.src_lo[1];
    b.src = make_rsrc(g.src_profile, (uint32_t)(sxn * syn * (g.src_hi[2] - g.src_lo[2])) * 4u);
    if constexpr (MS)
        b.msrc = make_rsrc(g.msrc_profile, (uint32_t)((g.msrc_hi[0] - g.msrc_lo[0]) * (g.msrc_hi[1] - g.msrc_lo[1]) *
                                                      (g.msrc_hi[2] - g.msrc_lo[2])) * 4u);

    // columns this thread touches: its own, one position of the LDS ring, one halo H cell
    c.own = make_col(g, c.x, c.y);
    c.rlx = c.rly = -1;
    c.ring.xy = -1;
    if (row == 0) { c.rlx = lane + 1; c.rly = 0; c.ring = make_col(g, c.i0 + lane, c.j0 - 1); }
    else if (row == 1) { c.rlx = lane + 1; c.rly = TY + 1; c.ring = make_col(g, c.i0 + lane, c.j0 + TY); }
    else if (row == 2 && lane < TY + 2) { c.rlx = 0; c.rly = lane; c.ring = make_col(g, c.i0 - 1, c.j0 - 1 + lane); }
    else if (row == 3 && lane < TY + 2) { c.rlx = EXT - 1; c.rly = lane; c.ring = make_col(g, c.i0 + TX, c.j0 - 1 + lane); }
    c.hex = c.hey = -1;
    c.hc.xy = -1;
    c.hc.x = c.hc.y = 0;
    c.hc.sx = c.hc.sy = -1;
    if (c.tid < TX + TY) {
        if (c.tid < TX) { c.hex = c.tid + 1; c.hey = 0; } else { c.hex = 0; c.hey = c.tid - TX + 1; }
        const int xr = c.i0 - 1 + c.hex, yr = c.j0 - 1 + c.hey;
        if (xr < g.nx && yr < g.ny) c.hc = make_col(g, xr, yr);   // positions past the far edge are never read
    }
    FwdLanes Ln;
    Ln.eo = lane_off(c.own.xy >= 0, c.own.xy);
    Ln.er = lane_off(c.ring.xy >= 0, c.ring.xy);
    Ln.o = lane_off(c.live, c.own.xy);
    Ln.hc = lane_off(c.hc.xy >= 0, c.hc.xy);
    Ln.src = lane_off(c.live && c.x >= g.src_lo[0] && c.x < g.src_hi[0] && c.y >= g.src_lo[1] && c.y < g.src_hi[1],
                      (c.x - g.src_lo[0]) + sxn * (c.y - g.src_lo[1]));
    Ln.m = box_lane(g.msrc_lo, g.msrc_hi, c.own);
    Ln.mh = box_lane(g.msrc_lo, g.msrc_hi, c.hc);
    Ln.po = psi_lane(g, c.own, c.live);
    Ln.ph = psi_lane(g, c.hc, c.hc.xy >= 0);
    Ln.ysl = c.own.sy >= 0;
    fill_coef_tile<TY, CZ>(g, ct, c.i0, c.j0, k0, c.tid, TX * TY);   // published by the prologue's barrier

    // the tile's class: the slabs that the cells it reads PML auxiliaries of reach
    // (own and halo columns, planes k0-1 .. k0+CZ-1; uniform over the block)
    const int sl = slab_class(g, c.i0 - 1, c.i0 + TX, c.j0 - 1, c.j0 + TY, k0 - 1, k0 + CZ);
    double e2;
    switch (sl) {
        case 0: e2 = fwd_tile<TY, CZ, MS, 0>(g, b, Ln, c, sE, sH, ct, k0, k1, wave, mwave); break;
        case 1: e2 = fwd_tile<TY, CZ, MS, 1>(g, b, Ln, c, sE, sH, ct, k0, k1, wave, mwave); break;
        case 2: e2 = fwd_tile<TY, CZ, MS, 2>(g, b, Ln, c, sE, sH, ct, k0, k1, wave, mwave); break;
        case 3: e2 = fwd_tile<TY, CZ, MS, 3>(g, b, Ln, c, sE, sH, ct, k0, k1, wave, mwave); break;
        case 4: e2 = fwd_tile<TY, CZ, MS, 4>(g, b, Ln, c, sE, sH, ct, k0, k1, wave, mwave); break;
        case 5: e2 = fwd_tile<TY, CZ, MS, 5>(g, b, Ln, c, sE, sH, ct, k0, k1, wave, mwave); break;
        case 6: e2 = fwd_tile<TY, CZ, MS, 6>(g, b, Ln, c, sE, sH, ct, k0, k1, wave, mwave); break;
        default: e2 = fwd_tile<TY, CZ, MS, 7>(g, b, Ln, c, sE, sH, ct, k0, k1, wave, mwave); break;
    }
    // detector partial of this tile (tiles intersecting the detector only; uniform per block)
    const int dx = tix - tl.dtx0, dy = tiy - tl.dty0, dz = tiz - tl.dtz0;
    if (dx < 0 || dy < 0 || dz < 0 || dx >= tl.dntx || dy >= tl.dnty || dz >= tl.dntz) return;
    for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off, 64);
    if (lane == 0) red[row] = e2;
    __syncthreads();
    if (c.tid == 0) {
        double sum = 0.0;
        for (int w = 0; w < TY; ++w) sum += red[w];
        partials[dx + (long long)tl.dntx * (dy + (long long)tl.dnty * dz)] = sum;
    }
}

// Recorder of one kept step (Section 2: the interface slices are recorded during the
// forward simulation): the tangential H^{n+1/2} of the three low faces (index P-1) and
// the tangential E^n of the three high faces (index n-P), each over the interior extent
// of its face, as the 12 blocks of kept step `slice`: encoded to the storage type, or
// (scaled FP8) in FP32 into the staging buffer that the two quantisation launches then
// encode.  E^n comes from the step's input buffer, H^{n+1/2} from its output buffer,
// or either from a buffer laid out as one kept step in FP32 (written by a two-step sweep,
// whose intermediate fields never reach a field buffer).  One thread per face cell and
// side, both tangential components.
template <int DT>
__global__ __launch_bounds__(256) void k_record(Grid g, const float* __restrict__ E, int e_mid,
                                                const float* __restrict__ H, int h_mid, void* __restrict__ dst) {
    const int face = g.my * g.mz + g.mx * g.mz + g.mx * g.my;   // < 2^31: 24 N < 2^31
    int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= 2 * face) return;
    const bool high = t >= face;
    if (high) t -= face;
    const FaceCell f = face_cell(g, t, high);
    const long long o0 = block_offset(g, f.blk) + f.u, o1 = block_offset(g, f.blk + 1) + f.u;
    float v0, v1;
    if (high ? e_mid : h_mid) {
        const float* A = high ? E : H;
        v0 = A[o0];
        v1 = A[o1];
    } else {
        const long long N = g.N;
        const float* A = high ? E : H + 3 * N;                 // E^n on the high faces, H^{n+1/2} on the low ones
        const long long idx = f.x + (long long)g.nx * (f.y + (long long)g.ny * f.z);
        v0 = A[f.c0 * N + idx];
        v1 = A[f.c1 * N + idx];
    }
    store_code<DT>(dst, o0, v0);
    store_code<DT>(dst, o1, v1);
}

// FP8 recorder of one kept step, in two launches over (chunk, block) grids so that
// every compute unit takes part: the absmax of each chunk of each (face,
// component) block of the FP32 staging copy (exact: max does not round), then
// per block the power-of-two scale from the chunks' maxima and the E4M3 codes.
// The chunk maxima sit after the staging values (REC_CHUNKS per block).
constexpr int REC_CHUNKS = 64;

__device__ inline void chunk_range(long long len, int chunks, int c, long long& lo, long long& hi) {
    const long long per = (len + chunks - 1) / chunks;
    lo = min(len, (long long)c * per);
    hi = min(len, lo + per);
}

__global__ __launch_bounds__(256) void k_rec_absmax(Grid g, const float* __restrict__ staging,
                                                    float* __restrict__ chunk_max, int chunks) {
    const int c = blockIdx.x, b = blockIdx.y;
    const long long off = block_offset(g, b);
    long long lo, hi;
    chunk_range(block_len(g, b), chunks, c, lo, hi);
    float m = 0.0f;
    for (long long t = lo + threadIdx.x; t < hi; t += 256) m = fmaxf(m, fabsf(staging[off + t]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) chunk_max[b * REC_CHUNKS + c] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_rec_encode(Grid g, const float* __restrict__ staging,
                                                    const float* __restrict__ chunk_max, int chunks,
                                                    void* __restrict__ store, int slice) {
    const int c = blockIdx.x, b = blockIdx.y;
    float mm = 0.0f;
    for (int i = 0; i < chunks; ++i) mm = fmaxf(mm, chunk_max[b * REC_CHUNKS + i]);
    const float sc = pow2f(fp8_scale_exp(mm));
    if (c == 0 && threadIdx.x == 0) ((float*)((char*)store + g.scale_off))[slice * 12 + b] = sc;
    const float inv = 1.0f / sc;   // exact: sc is a power of two in the normal range
    const long long off = block_offset(g, b);
    long long lo, hi;
    chunk_range(block_len(g, b), chunks, c, lo, hi);
    uint8_t* q = (uint8_t*)store + (long long)slice * g.slice_stride + off;
    for (long long t = lo + threadIdx.x; t < hi; t += 256) q[t] = enc_e4m3(staging[off + t] * inv);
}

// Fixed-order FP64 reduction of the detector partials: per-step terms, then their sum.
__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ partials, int steps, int per_step,
                                                    double* __restrict__ loss, double* __restrict__ series) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int n = threadIdx.x; n < steps; n += 256) {
        double s = 0.0;
        const double* p = partials + (long long)n * per_step;
        for (int t = 0; t < per_step; ++t) s += p[t];
        if (series) series[n] = s;
        acc += s;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0];
}

template <int TY, int CZ>
static void launch_fwd_step_t(const Grid& g, const Tiling& t, const float* F0, float* F1, float* psi, int hcopy,
                              const float* eps, float wave, float mwave, double* partials, const RecJob* job,
                              hipStream_t s) {
    RecJob j{};
    long long extra = 0;
    if (job && g.P > 0 && g.vps > 0 && (job->dst_e || job->dst_h)) {
        j = *job;
        extra = (g.vps / 2 + TX * TY - 1) / (TX * TY);   // one thread per face cell and side
    }
    const dim3 grid((unsigned)(t.count + extra)), block(TX, TY);
    if (g.msrc_hi[0] > g.msrc_lo[0])
        launch_kernel(K_FWD_STEP, k_fwd_step<TY, CZ, true>, grid, block, s, g, t, F0, F1, psi, hcopy, eps, wave,
                      mwave, partials, j);
    else
        launch_kernel(K_FWD_STEP, k_fwd_step<TY, CZ, false>, grid, block, s, g, t, F0, F1, psi, hcopy, eps, wave,
                      mwave, partials, j);
}

void launch_fwd_step(const Grid& g, const Tiling& t, const float* F0, float* F1, float* psi, int hcopy,
                     const float* eps, float wave, float mwave, double* partials, const RecJob* job, hipStream_t s) {
    if (t.ty == 4 && t.cz == 4) launch_fwd_step_t<4, 4>(g, t, F0, F1, psi, hcopy, eps, wave, mwave, partials, job, s);
    else if (t.ty == 4) launch_fwd_step_t<4, 8>(g, t, F0, F1, psi, hcopy, eps, wave, mwave, partials, job, s);
    else if (t.cz == 4) launch_fwd_step_t<8, 4>(g, t, F0, F1, psi, hcopy, eps, wave, mwave, partials, job, s);
    else launch_fwd_step_t<8, 8>(g, t, F0, F1, psi, hcopy, eps, wave, mwave, partials, job, s);
}

void launch_record_job(const Grid& g, const RecJob& job, hipStream_t s) {
    if (g.P == 0 || g.vps == 0 || (!job.dst_e && !job.dst_h)) return;
    const long long n = g.vps / 2;
    launch_kernel(K_RECORD, k_record_job, dim3((unsigned)((n + 255) / 256)), dim3(256), s, g, job);
}

void launch_record(const Grid& g, const float* E, bool e_mid, const float* H, bool h_mid, void* store,
                   float* staging, int slice, hipStream_t s) {
    if (g.P == 0 || g.vps == 0) return;
    const long long n = g.vps / 2;                      // face cells on both sides
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    void* dst = g.dtype == 3 ? (void*)staging : (void*)((char*)store + slice * g.slice_stride);
    with_dtype(g.dtype, [&]<int DT>() {
        launch_kernel(K_RECORD, k_record<DT>, grid, block, s, g, E, (int)e_mid, H, (int)h_mid, dst);
    });
}

long long rec_quant_scratch_floats(const Grid& g) {
    return ((g.vps + 63) / 64) * 64 + 12 * REC_CHUNKS;
}

void launch_rec_quant(const Grid& g, const float* staging, void* store, int slice, hipStream_t s) {
    long long longest = 0;
    for (int b = 0; b < 12; ++b) longest = std::max(longest, (long long)block_len(g, b));
    const int chunks = (int)std::min<long long>(REC_CHUNKS, std::max<long long>(1, (longest + 2047) / 2048));
    float* chunk_max = const_cast<float*>(staging) + ((g.vps + 63) / 64) * 64;
    launch_kernel(K_REC_QUANT, k_rec_absmax, dim3(chunks, 12), dim3(256), s, g, staging, chunk_max, chunks);
    launch_kernel(K_REC_QUANT, k_rec_encode, dim3(chunks, 12), dim3(256), s, g, staging, chunk_max, chunks, store,
                  slice);
}

void launch_loss_final(const double* partials, int steps, int per_step, double* loss, double* series,
                       hipStream_t s) {
    launch_kernel(K_LOSS_FINAL, k_loss_final, dim3(1), dim3(256), s, partials, steps, per_step, loss, series);
}

// ----------------------------------------------------------------------------
// Standalone codec round trip (same encoders as the recorder)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_codec_roundtrip(int dtype, const float* __restrict__ x, long long len,
                                                         void* __restrict__ codes, float* __restrict__ scales,
                                                         float* __restrict__ out) {
    const long long b = blockIdx.x;
    const float* xb = x + b * len;
    float* ob = out + b * len;
    if (dtype == 3) {
        float m = 0.0f;
        for (long long t = threadIdx.x; t < len; t += 256) m = fmaxf(m, fabsf(xb[t]));
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        __shared__ float red[4];
        __shared__ float sc;
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            sc = pow2f(fp8_scale_exp(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
            scales[b] = sc;
        }
        __syncthreads();
        const float inv = 1.0f / sc;
        uint8_t* q = (uint8_t*)codes + b * len;
        for (long long t = threadIdx.x; t < len; t += 256) {
            uint8_t c = enc_e4m3(xb[t] * inv);
            q[t] = c;
            ob[t] = dec_e4m3(c) * sc;
        }
        return;
    }
    for (long long t = threadIdx.x; t < len; t += 256) {
        float v = xb[t];
        if (dtype == 0) {
            ((float*)codes)[b * len + t] = v;
            ob[t] = v;
        } else if (dtype == 1) {
            uint16_t c = enc_fp16(v);
            ((uint16_t*)codes)[b * len + t] = c;
            ob[t] = dec_fp16(c);
        } else if (dtype == 2) {
            uint16_t c = enc_bf16(v);
            ((uint16_t*)codes)[b * len + t] = c;
            ob[t] = dec_bf16(c);
        } else {
            uint8_t c = enc_unscaled(dtype, v);
            ((uint8_t*)codes)[b * len + t] = c;
            ob[t] = dec_unscaled(dtype, c);
        }
    }
}

void launch_codec_roundtrip(int dtype, const float* values, long long n_blocks, long long block_len,
                            void* codes, float* scales, float* decoded, hipStream_t s) {
    if (n_blocks <= 0) return;
    launch_kernel(K_CODEC, k_codec_roundtrip, dim3((unsigned)n_blocks), dim3(256), s, dtype, values, block_len,
                       codes, scales, decoded);
}

}  // namespace fdtd
