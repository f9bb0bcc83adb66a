// Time-reversed gradient pass (gfx950).
//
// Reverse step n (n = T-1 .. 0) undoes forward step n in two fused sweeps,
// each with the shape of a forward step (see march.h):
//
//   prim_rev  the primal state backwards through the lossless interior I
//             (every interior node has PML depth 0, so there is no PML term):
//               E^n       = E^{n+1} - (dt/eps)(curl H^{n+1/2} - J^n)   on I,
//                           E^n on the high interface faces from the store,
//               H^{n-1/2} = H^{n+1/2} + dt curl E^n                    on I,
//                           H^{n-1/2} on the low interface faces from the store
//             (Section 1: backwards from the final step; Section 2: the
//             recorded interface fields act as sources), and the gradient
//               epsbar -= (dt/eps^2) sum_c Ebar_c (U_c - J_c)   on the design box (FP64),
//             with Ebar including this step's loss seed 2 E^{n+1} on the detector.
//             It sweeps I plus its one-cell shell only.
//
//   adj       the exact transpose of forward step n over the whole grid, PML
//             included, for the adjoint state (Ebar, Hbar) and its PML
//             auxiliaries:
//               seed    Ebar += 2 E^{n+1} on the detector,
//               E half  v = (dt/eps) Ebar; per E-half term t = (c, d, s, f):
//                       P = psibar_t + s v_c, gbar = s kinv_E v_c + a_E P, psibar_t <- b_E P,
//                       Hbar_f += gbar(p) - gbar(p + e_d),
//               H half  w = -dt Hbar; per H-half term t:
//                       P = psibar_t + s w_c, gbar = s kinv_H w_c + a_H P, psibar_t <- b_H P,
//                       Ebar_f += gbar(p - e_d) - gbar(p).
//
// Both sweeps read one buffer and write the other (primal, adjoint and PML
// auxiliaries all ping-pong), so the gradient of step n reads the adjoint
// state before step n's transpose and the seed reads E^{n+1} before it is
// replaced.
//
// The interface shell that prim_rev of step n-1 needs (E^{n-1} on the high
// faces, H^{n-3/2} on the low ones, decoded and interpolated from the store) is
// written by extra workgroups appended to the adjoint launch of step n, which
// touches no primal buffer: E^{n-1} into the buffer prim_rev of step n has just
// written (the input of step n-1, whose high-face E positions no sweep reads
// otherwise, so that prim_rev reads E^{n} and the shell with one load), H^{n-3/2}
// into the buffer prim_rev of step n has just read (the output of step n-1).  Only
// the first reverse step needs a launch of its own.
// Stores carry device scope (cache-policy bit sc1), as in the forward sweep: they
// write through the XCD's L2 instead of leaving dirty lines for the writeback at
// the end of every launch (measured: about 3 us of 64 per reverse step at 128^3).
#ifndef FDTD_REV_ST_AUX
#define FDTD_REV_ST_AUX 16
#endif
#define FDTD_ST_AUX FDTD_REV_ST_AUX
#include "march.h"

namespace fdtd {

// --------------------------------------------------------------------------
// adjoint sweep
// --------------------------------------------------------------------------

// Transpose of one half step's CPML at one cell, on the axes of tile class SL.  o holds
// the six raw terms (s * v_c for the E half, s * w_c for the H half; x: 3, 4; y: 0, 5;
// z: 1, 2); inside the slab of a term's axis P = psibar + o, o <- kinv o + a P and the
// new auxiliary is b P.  Outside a slab the coefficients (0, 0, 1) leave o unchanged;
// the axes outside SL have them at every cell of the tile (new auxiliary 0, never stored).
template <int SL>
__device__ inline void gbar_axes(const Cf& cx, const Cf& cy, const Cf& cz, float o[6], const float pin[6],
                                 float pout[6]) {
    float q;
    pout[0] = pout[1] = pout[2] = pout[3] = pout[4] = pout[5] = 0.0f;
    if constexpr ((SL & 1) != 0) {
        q = pin[3] + o[3]; o[3] = cx.k * o[3] + cx.a * q; pout[3] = cx.b * q;
        q = pin[4] + o[4]; o[4] = cx.k * o[4] + cx.a * q; pout[4] = cx.b * q;
    }
    if constexpr ((SL & 2) != 0) {
        q = pin[0] + o[0]; o[0] = cy.k * o[0] + cy.a * q; pout[0] = cy.b * q;
        q = pin[5] + o[5]; o[5] = cy.k * o[5] + cy.a * q; pout[5] = cy.b * q;
    }
    if constexpr ((SL & 4) != 0) {
        q = pin[1] + o[1]; o[1] = cz.k * o[1] + cz.a * q; pout[1] = cz.b * q;
        q = pin[2] + o[2]; o[2] = cz.k * o[2] + cz.a * q; pout[2] = cz.b * q;
    }
}

// Hbar after the E-half transpose at the cell of extended coordinates (ex, ey):
// Hbar0 + sum_t (gbar_t(p) - gbar_t(p + e_d)), +z from the next plane.
template <int TY>
__device__ inline void hbar_new(const float (*cur)[TY + 2][EXT], const float (*nxt)[TY + 2][EXT], int ex, int ey,
                                const float h0[3], float h[3]) {
    h[0] = h0[0] + (cur[2][ey][ex] - nxt[2][ey][ex]) + (cur[5][ey][ex] - cur[5][ey + 1][ex]);
    h[1] = h0[1] + (cur[1][ey][ex] - nxt[1][ey][ex]) + (cur[4][ey][ex] - cur[4][ey][ex + 1]);
    h[2] = h0[2] + (cur[0][ey][ex] - cur[0][ey + 1][ex]) + (cur[3][ey][ex] - cur[3][ey][ex + 1]);
}

// Tiles that reach no PML slab (class 0) keep three values per cell in the LDS planes
// instead of six: the E-half terms there are (vx, -vx, vy, -vy, vz, -vz), kept as vx, vy,
// vz in slots 0-2, and the H-half terms (-w0, w0, -w1, w1, -w2, w2), w = dt Hbar, kept as
// w0, w1, w2.  The sums read them back with the same signs, so the results are the same
// bits as with all six.
template <int TY, int SL>
__device__ __forceinline__ void put_g(float (*p)[TY + 2][EXT], int y, int x, const float o[6]) {
    if constexpr (SL == 0) {
        p[0][y][x] = o[0]; p[1][y][x] = o[2]; p[2][y][x] = o[4];
    } else {
        #pragma unroll
        for (int t = 0; t < 6; ++t) p[t][y][x] = o[t];
    }
}

template <int TY, int SL>
__device__ __forceinline__ void put_gh(float (*p)[TY + 1][TX + 1], int y, int x, const float o[6]) {
    if constexpr (SL == 0) {
        p[0][y][x] = o[1]; p[1][y][x] = o[3]; p[2][y][x] = o[5];
    } else {
        #pragma unroll
        for (int t = 0; t < 6; ++t) p[t][y][x] = o[t];
    }
}

template <int TY, int SL>
__device__ __forceinline__ void hbar_new_s(const float (*cur)[TY + 2][EXT], const float (*nxt)[TY + 2][EXT], int ex,
                                           int ey, const float h0[3], float h[3]) {
    if constexpr (SL == 0) {
        h[0] = h0[0] + (cur[1][ey][ex] - nxt[1][ey][ex]) + ((-cur[2][ey][ex]) - (-cur[2][ey + 1][ex]));
        h[1] = h0[1] + ((-cur[0][ey][ex]) - (-nxt[0][ey][ex])) + (cur[2][ey][ex] - cur[2][ey][ex + 1]);
        h[2] = h0[2] + (cur[0][ey][ex] - cur[0][ey + 1][ex]) + ((-cur[1][ey][ex]) - (-cur[1][ey][ex + 1]));
    } else {
        hbar_new<TY>(cur, nxt, ex, ey, h0, h);
    }
}

struct AdjBufs {
    rsrc_t A0, A1, eps, psi;   // adjoint fields in / out (Ebar then Hbar), both PML copies
    uint32_t pin, pout;        // byte offsets of the PML copies in / out
};

// Loop-invariant per-lane byte offsets of the adjoint sweep: Ebar/eps of the own column
// (boundary rule) and of the ring position, the own cell (live lanes), the halo cell,
// and the PML auxiliaries of the own column (boundary rule and live), ring and halo.
struct AdjLanes {
    uint32_t eo, er, o, hc;
    PsiLane pg, po, pr, ph;
    bool ysl;                 // the own row lies in a y slab (uniform across a wave)
};

// What the adjoint sweep reads from memory for plane k of its column, loaded
// one plane ahead: Ebar (loss seed included), eps and the E-side auxiliaries at
// plane k+1 for the own cell and the LDS-ring position; Hbar and the H-side
// auxiliaries at plane k for the own cell and the halo cell.
struct AdjIn {
    float eb[3], ep, pe[6];
    float rb[3], rep, rpe[6];
    float hb[3], ph[6];
    float hhb[3], phh[6];
};

// Ebar, eps and E-side auxiliaries at the lane offsets (v, pl) on plane z (z < 0: 0, eps 1).
template <int SL>
__device__ __forceinline__ void load_ge_in(const Grid& g, const AdjBufs& b, uint32_t v, const PsiLane& pl, int z,
                                           int plane, uint32_t nb, float eb[3], float& ep, float pe[6]) {
    const uint32_t s = uni(z < 0 ? 0u : (uint32_t)(z * plane) << 2);
    const uint32_t vv = z < 0 ? OOB : v;
    bld3v(b.A0, vv, s, nb, eb);
    const float e = bldv(b.eps, vv, s);
    ep = e == 0.0f ? 1.0f : e;          // outside the domain eps reads 0
    PsiPlane pp = psi_plane(g, 1, z < 0 ? 0 : z, b.pin);
    pp.zs = pp.zs && z >= 0;
    PsiLane l = pl;
    if (z < 0) l.x = l.y = l.z = OOB;
    bld_psi_s<SL>(b.psi, l, pp, pe);
}

template <int TY, int SL>
__device__ __forceinline__ void load_adj_in(const Grid& g, const AdjBufs& b, const AdjLanes& L, const FwdCtx<TY>& c,
                                            int k, AdjIn& d) {
    const uint32_t nb = (uint32_t)c.N << 2;
    const int z1 = bound(k + 1, g.nz, g.periodic);
    load_ge_in<SL>(g, b, L.eo, L.pg, z1, c.plane, nb, d.eb, d.ep, d.pe);
    load_ge_in<SL>(g, b, L.er, L.pr, z1, c.plane, nb, d.rb, d.rep, d.rpe);
    const uint32_t sk = uni(((uint32_t)(k * c.plane) << 2) + 3 * nb);
    bld3v(b.A0, L.o, sk, nb, d.hb);
    bld3v(b.A0, L.hc, sk, nb, d.hhb);
    const PsiPlane pH = psi_plane(g, 0, k, b.pin);
    bld_psi_s<SL>(b.psi, L.po, pH, d.ph);
    bld_psi_s<SL>(b.psi, L.ph, pH, d.phh);
}

// E-half gbar at one position from its inputs: v = (dt/eps) Ebar, raw terms
// (vx, -vx, vy, -vy, vz, -vz), CPML transpose on the axes of class SL; the new
// auxiliaries go to pout.
template <int SL>
__device__ __forceinline__ void ge_terms(float dt, const float eb[3], float ep, const float pe[6], const Cf& cx,
                                         const Cf& cy, const Cf& cz, float o[6], float pout[6]) {
    const float cc = dt_over_eps(dt, ep);
    const float vx = cc * eb[0], vy = cc * eb[1], vz = cc * eb[2];
    o[0] = vx; o[1] = -vx; o[2] = vy; o[3] = -vy; o[4] = vz; o[5] = -vz;
    gbar_axes<SL>(cx, cy, cz, o, pe, pout);
}

// Transpose of one axis' CPML on its two terms (x: 3, 4; y: 0, 5; z: 1, 2):
// q = psibar + o, o <- kinv o + a q, new psibar = b q.
__device__ inline void gbar_axis(const Cf& c, int i, int j, float o[6], const float pin[6], float pout[6]) {
    float q = pin[i] + o[i];
    o[i] = c.k * o[i] + c.a * q;
    pout[i] = c.b * q;
    q = pin[j] + o[j];
    o[j] = c.k * o[j] + c.a * q;
    pout[j] = c.b * q;
}

// E-half gbar of the own cell at plane k+1 (y and z parts under uniform branches; the
// axes outside class SL not at all).
template <int TY, int CZ, int SL>
__device__ __forceinline__ void ge_own(float dt, const CoefTile<TY, CZ>& ct, int lx, int ly, int lz, bool ysl,
                                       bool zsl, const float eb[3], float ep, const float pe[6], float o[6],
                                       float po[6]) {
    const float cc = dt_over_eps(dt, ep);
    const float vx = cc * eb[0], vy = cc * eb[1], vz = cc * eb[2];
    o[0] = vx; o[1] = -vx; o[2] = vy; o[3] = -vy; o[4] = vz; o[5] = -vz;
    po[0] = po[1] = po[2] = po[3] = po[4] = po[5] = 0.0f;
    if constexpr ((SL & 1) != 0) gbar_axis(cf_x(ct, 0, lx), 3, 4, o, pe, po);
    if constexpr ((SL & 2) != 0) { if (ysl) gbar_axis(cf_y(ct, 0, ly), 0, 5, o, pe, po); }
    if constexpr ((SL & 4) != 0) { if (zsl) gbar_axis(cf_z(ct, 0, lz), 1, 2, o, pe, po); }
}

// One plane k of the adjoint sweep: E-half gbar of plane k+1 (own cell and ring
// position) into LDS, the H-half transpose on the own and halo cells of plane k,
// then Ebar of the own cell at plane k.
template <int TY, int CZ, int SL>
__device__ __forceinline__ void adj_plane(const Grid& g, const AdjBufs& b, const AdjLanes& L, const FwdCtx<TY>& c,
                                          float (*sG)[6][TY + 2][EXT], float (*sGH)[TY + 1][TX + 1],
                                          const CoefTile<TY, CZ>& ct, int kk, int k, bool own_next, int cur,
                                          const AdjIn& in, float ebc[3], float& g1p, float& g2p) {
    const int nxt = 1 - cur;
    const int row = c.row, lane = c.lane;
    const uint32_t nb = (uint32_t)c.N << 2;
    const float dt = g.dt;
    const int z1 = bound(k + 1, g.nz, g.periodic);
    // ---- E-half gbar of plane k+1 ----
    {
        PsiPlane pp = psi_plane(g, 1, z1 < 0 ? 0 : z1, b.pout);
        pp.zs = pp.zs && z1 >= 0;
        float o[6], po[6];
        ge_own<TY, CZ, SL>(dt, ct, lane + 1, row + 1, kk + 2, L.ysl, pp.zs, in.eb, in.ep, in.pe, o, po);
        put_g<TY, SL>(sG[nxt], row + 1, lane + 1, o);
        PsiLane l = L.po;                        // the block's own cells at k+1 only
        if (!own_next || z1 < 0) l.x = l.y = l.z = OOB;
        bst_psi_s<SL>(b.psi, l, pp, po);
        if (c.rlx >= 0) {
            ge_terms<SL>(dt, in.rb, in.rep, in.rpe, cf_x(ct, 0, c.rlx), cf_y(ct, 0, c.rly), cf_z(ct, 0, kk + 2), o,
                         po);
            put_g<TY, SL>(sG[nxt], c.rly, c.rlx, o);
        }
    }
    __syncthreads();
    // ---- H-half transpose at plane k: own cell (stored) and halo cell (LDS only) ----
    const uint32_t sk = uni((uint32_t)(k * c.plane) << 2);
    const PsiPlane pH = psi_plane(g, 0, k, b.pout);
    float og[6];
    {
        float h[3], po[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        hbar_new_s<TY, SL>(sG[cur], sG[nxt], lane + 1, row + 1, in.hb, h);
        bst3v(b.A1, L.o, sk + 3 * nb, nb, h);
        og[0] = -dt * h[0]; og[1] = dt * h[0]; og[2] = -dt * h[1]; og[3] = dt * h[1]; og[4] = -dt * h[2];
        og[5] = dt * h[2];
        if constexpr ((SL & 1) != 0) gbar_axis(cf_x(ct, 1, lane + 1), 3, 4, og, in.ph, po);
        if constexpr ((SL & 2) != 0) { if (L.ysl) gbar_axis(cf_y(ct, 1, row + 1), 0, 5, og, in.ph, po); }
        if constexpr ((SL & 4) != 0) { if (pH.zs) gbar_axis(cf_z(ct, 1, kk + 1), 1, 2, og, in.ph, po); }
        if (!c.live) og[0] = og[1] = og[2] = og[3] = og[4] = og[5] = 0.0f;
        bst_psi_s<SL>(b.psi, L.po, pH, po);
        put_gh<TY, SL>(sGH, row + 1, lane + 1, og);
    }
    if (c.hex >= 0) {
        float o[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (c.hc.xy >= 0) {
            float h[3], po[6];
            hbar_new_s<TY, SL>(sG[cur], sG[nxt], c.hex, c.hey, in.hhb, h);
            o[0] = -dt * h[0]; o[1] = dt * h[0]; o[2] = -dt * h[1]; o[3] = dt * h[1]; o[4] = -dt * h[2];
            o[5] = dt * h[2];
            gbar_axes<SL>(cf_x(ct, 1, c.hex), cf_y(ct, 1, c.hey), cf_z(ct, 1, kk + 1), o, in.phh, po);
        }
        put_gh<TY, SL>(sGH, c.hey, c.hex, o);
    }
    __syncthreads();
    // ---- Ebar at plane k: Ex <- terms 2 (z), 5 (y); Ey <- 1 (z), 4 (x); Ez <- 0 (y), 3 (x) ----
    float e[3];
    if constexpr (SL == 0) {   // slots w0, w1, w2: term 5 = w2, 4 = -w2, 0 = -w0, 3 = w1
        e[0] = ebc[0] + (g2p - og[2]) + (sGH[2][row][lane + 1] - og[5]);
        e[1] = ebc[1] + (g1p - og[1]) + ((-sGH[2][row + 1][lane]) - og[4]);
        e[2] = ebc[2] + ((-sGH[0][row][lane + 1]) - og[0]) + (sGH[1][row + 1][lane] - og[3]);
    } else {
        e[0] = ebc[0] + (g2p - og[2]) + (sGH[5][row][lane + 1] - og[5]);
        e[1] = ebc[1] + (g1p - og[1]) + (sGH[4][row + 1][lane] - og[4]);
        e[2] = ebc[2] + (sGH[0][row][lane + 1] - og[0]) + (sGH[3][row + 1][lane] - og[3]);
    }
    bst3v(b.A1, L.o, sk, nb, e);
    g1p = og[1];
    g2p = og[2];
    ebc[0] = in.eb[0]; ebc[1] = in.eb[1]; ebc[2] = in.eb[2];
}

// The interface shell of one reverse step written into a field buffer (E then H)
// from the store: H at the low faces (blocks 0-5, interpolation qH) when do_h, E at
// the high faces (blocks 6-11, interpolation qE) when do_e.  One thread t per face
// cell and side (2 (my mz + mx mz + mx my) in all); the first ax+ay+az threads take
// the low faces.
template <int DT>
__device__ inline void shell_cell(const Grid& g, const ShellJob& j, int t) {
    const int face = g.my * g.mz + g.mx * g.mz + g.mx * g.my;   // < 2^31: 24 N < 2^31
    const bool high = t >= face;
    if (high) t -= face;
    if (t >= face || (high ? !j.do_e : !j.do_h)) return;
    const FaceCell f = face_cell(g, t, high);
    const Interp& q = high ? j.qE : j.qH;
    const float v0 = shell_value_t<DT>(g, j.store, q, f.blk, f.u), v1 = shell_value_t<DT>(g, j.store, q, f.blk + 1, f.u);
    if (j.slice) {                                            // one kept step's layout, both sides in FE
        j.FE[block_offset(g, f.blk) + f.u] = v0;
        j.FE[block_offset(g, f.blk + 1) + f.u] = v1;
        return;
    }
    const long long N = g.N;
    float* A = high ? j.FE : j.FH + 3 * N;                    // E for the high faces, H for the low ones
    // an x-face cell (y, z) one per row of its plane would cost a partial-line write per
    // value; with xrow it goes to position y - P of row 0 of plane z instead (PML cells
    // that the one-step reversal never reads otherwise), where a wave writes it contiguously
    const long long idx = (j.xrow && f.blk % 6 == 0) ? (f.y - g.P) + (long long)g.nx * g.ny * f.z
                                                    : f.x + (long long)g.nx * (f.y + (long long)g.ny * f.z);
    A[f.c0 * N + idx] = v0;
    A[f.c1 * N + idx] = v1;
}

// the storage type is uniform over the launch: one branch per wave
__device__ inline void shell_cell_any(const Grid& g, const ShellJob& j, int t) {
    switch (g.dtype) {
        case 0: shell_cell<0>(g, j, t); break;
        case 1: shell_cell<1>(g, j, t); break;
        case 2: shell_cell<2>(g, j, t); break;
        case 3: shell_cell<3>(g, j, t); break;
        case 4: shell_cell<4>(g, j, t); break;
        case 5: shell_cell<5>(g, j, t); break;
        case 6: shell_cell<6>(g, j, t); break;
        case 7: shell_cell<7>(g, j, t); break;
        case 8: shell_cell<8>(g, j, t); break;
        default: shell_cell<9>(g, j, t); break;
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_inject_shell(Grid g, ShellJob j) {
    shell_cell<DT>(g, j, (int)blockIdx.x * 256 + (int)threadIdx.x);
}

// The z-march of one adjoint tile of class SL (slab_class) over planes [k0, k1).
template <int TY, int CZ, int SL>
__device__ __forceinline__ void adj_tile(const Grid& g, const AdjBufs& b, const AdjLanes& Ln, const FwdCtx<TY>& c,
                                         float (*sG)[6][TY + 2][EXT], float (*sGH)[TY + 1][TX + 1],
                                         const CoefTile<TY, CZ>& ct, int k0, int k1) {
    const int lane = c.lane, row = c.row;
    const uint32_t nb = (uint32_t)c.N << 2;
    const float dt = g.dt;
    // prologue: E-half gbar of planes k0-1 and k0, Ebar of the own cell at k0, and the
    // z-terms of the H-half gbar of the own cell at k0-1
    AdjIn pin[2];
    float ebc[3];
    float g1p, g2p;
    {
        const int zm = bound(k0 - 1, g.nz, g.periodic);
        const int z0 = bound(k0, g.nz, g.periodic);
        float eb[3], ep, pe[6], rb[3], rep, rpe[6], eb0[3], ep0, pe0[6], rb0[3], rep0, rpe0[6], hb[3], ph[6];
        load_ge_in<SL>(g, b, Ln.eo, Ln.pg, zm, c.plane, nb, eb, ep, pe);
        load_ge_in<SL>(g, b, Ln.er, Ln.pr, zm, c.plane, nb, rb, rep, rpe);
        load_ge_in<SL>(g, b, Ln.eo, Ln.pg, z0, c.plane, nb, eb0, ep0, pe0);
        load_ge_in<SL>(g, b, Ln.er, Ln.pr, z0, c.plane, nb, rb0, rep0, rpe0);
        const bool pro = c.live && zm >= 0;
        const uint32_t sm = uni(zm < 0 ? 0u : ((uint32_t)(zm * c.plane) << 2) + 3 * nb);
        bld3v(b.A0, zm < 0 ? OOB : Ln.o, sm, nb, hb);
        PsiPlane pm = psi_plane(g, 0, zm < 0 ? 0 : zm, b.pin);
        pm.zs = pm.zs && zm >= 0;
        PsiLane lm = Ln.po;
        if (zm < 0) lm.x = lm.y = lm.z = OOB;
        bld_psi_s<SL>(b.psi, lm, pm, ph);
        load_adj_in<TY, SL>(g, b, Ln, c, k0, pin[0]);
        float o[6], po[6];
        ge_terms<SL>(dt, eb, ep, pe, cf_x(ct, 0, lane + 1), cf_y(ct, 0, row + 1), cf_z(ct, 0, 0), o, po);
        put_g<TY, SL>(sG[0], row + 1, lane + 1, o);
        ge_terms<SL>(dt, eb0, ep0, pe0, cf_x(ct, 0, lane + 1), cf_y(ct, 0, row + 1), cf_z(ct, 0, 1), o, po);
        put_g<TY, SL>(sG[1], row + 1, lane + 1, o);
        // the own cell's E-side auxiliaries at k0 belong to this block
        bst_psi_s<SL>(b.psi, Ln.po, psi_plane(g, 1, z0, b.pout), po);
        if (c.rlx >= 0) {
            ge_terms<SL>(dt, rb, rep, rpe, cf_x(ct, 0, c.rlx), cf_y(ct, 0, c.rly), cf_z(ct, 0, 0), o, po);
            put_g<TY, SL>(sG[0], c.rly, c.rlx, o);
            ge_terms<SL>(dt, rb0, rep0, rpe0, cf_x(ct, 0, c.rlx), cf_y(ct, 0, c.rly), cf_z(ct, 0, 1), o, po);
            put_g<TY, SL>(sG[1], c.rly, c.rlx, o);
        }
        ebc[0] = eb0[0]; ebc[1] = eb0[1]; ebc[2] = eb0[2];
        __syncthreads();
        float h[3];
        hbar_new_s<TY, SL>(sG[0], sG[1], lane + 1, row + 1, hb, h);
        o[0] = -dt * h[0]; o[1] = dt * h[0]; o[2] = -dt * h[1]; o[3] = dt * h[1]; o[4] = -dt * h[2]; o[5] = dt * h[2];
        gbar_axes<SL>(cf_x(ct, 1, lane + 1), cf_y(ct, 1, row + 1), cf_z(ct, 1, 0), o, ph, po);
        g1p = pro ? o[1] : 0.0f;
        g2p = pro ? o[2] : 0.0f;
    }
    __syncthreads();   // the first plane overwrites sG[0], which the prologue has just read
    #pragma unroll
    for (int kk = 0; kk < CZ; ++kk) {
        const int k = k0 + kk;
        if (kk + 1 < CZ) load_adj_in<TY, SL>(g, b, Ln, c, min(k + 1, g.nz - 1), pin[(kk + 1) & 1]);
        if (k < k1)
            adj_plane<TY, CZ, SL>(g, b, Ln, c, sG, sGH, ct, kk, k, k + 1 < k1, (kk + 1) & 1, pin[kk & 1], ebc, g1p, g2p);
    }
}

// One adjoint step: (Ebar, Hbar) in A0 and the auxiliaries in PML copy `pcopy` ->
// A1 and copy 1 - pcopy.  Ebar already carries this step's loss seed (added by the
// primal reversal).  Unrolled over the CZ planes and software-pipelined like the
// forward sweep; each block runs the code of its tile's class, as the forward sweep
// does.  Workgroups past the tile count write the shell `job`.
#ifndef FDTD_ADJ_WAVES
#define FDTD_ADJ_WAVES 1
#endif
template <int TY, int CZ>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(FDTD_ADJ_WAVES))) void k_adj_step(
    Grid g, Tiling tl, const float* __restrict__ A0, float* __restrict__ A1, const float* __restrict__ eps,
    float* __restrict__ psi, int pcopy, ShellJob job) {
    __shared__ float sG[2][6][TY + 2][EXT];
    __shared__ float sGH[6][TY + 1][TX + 1];
    __shared__ CoefTile<TY, CZ> ct;
    if ((int)blockIdx.x >= tl.count) {   // trailing workgroups: the next reverse step's interface shell
        shell_cell_any(g, job, ((int)blockIdx.x - tl.count) * (TX * TY) + (int)(threadIdx.y * TX + threadIdx.x));
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
    const int lane = c.lane, row = c.row;
    AdjBufs b;
    const uint32_t psib = (uint32_t)g.psi_total * 4u;
    b.A0 = make_rsrc(A0, (uint32_t)(6 * c.N) * 4u);
    b.A1 = make_rsrc(A1, (uint32_t)(6 * c.N) * 4u);
    b.eps = make_rsrc(eps, (uint32_t)(c.plane * g.nz) * 4u);
    b.psi = make_rsrc(psi, 2 * psib);
    b.pin = pcopy ? psib : 0u;
    b.pout = pcopy ? 0u : psib;

    c.own = make_col(g, c.x, c.y);
    c.rlx = c.rly = -1;
    c.ring.xy = -1;
    c.ring.x = c.ring.y = 0;
    c.ring.sx = c.ring.sy = -1;
    if (row == 0) { c.rlx = lane + 1; c.rly = 0; c.ring = make_col(g, c.i0 + lane, c.j0 - 1); }
    else if (row == 1) { c.rlx = lane + 1; c.rly = TY + 1; c.ring = make_col(g, c.i0 + lane, c.j0 + TY); }
    else if (row == 2 && lane < TY + 2) { c.rlx = 0; c.rly = lane; c.ring = make_col(g, c.i0 - 1, c.j0 - 1 + lane); }
    else if (row == 3 && lane < TY + 2) { c.rlx = EXT - 1; c.rly = lane; c.ring = make_col(g, c.i0 + TX, c.j0 - 1 + lane); }
    c.hex = c.hey = -1;
    c.hc.xy = -1;
    c.hc.x = c.hc.y = 0;
    c.hc.sx = c.hc.sy = -1;
    // the halo cells: on waves 4-5 of an 8-row tile, so that no wave holds both ring and
    // halo work (512x512x256: 916.8 -> 912.4 us), on waves 0-1 of a 4-row one
    const int ht = TY == 8 ? c.tid - 4 * TX : c.tid;
    if (ht >= 0 && ht < TX + TY) {
        if (ht < TX) { c.hex = ht + 1; c.hey = 0; } else { c.hex = 0; c.hey = ht - TX + 1; }
        const int xr = c.i0 - 1 + c.hex, yr = c.j0 - 1 + c.hey;
        if (xr < g.nx && yr < g.ny) c.hc = make_col(g, xr, yr);
    }
    AdjLanes Ln;
    Ln.eo = lane_off(c.own.xy >= 0, c.own.xy);
    Ln.er = lane_off(c.ring.xy >= 0, c.ring.xy);
    Ln.o = lane_off(c.live, c.own.xy);
    Ln.hc = lane_off(c.hc.xy >= 0, c.hc.xy);
    Ln.pg = psi_lane(g, c.own, c.own.xy >= 0);
    Ln.po = psi_lane(g, c.own, c.live);
    Ln.pr = psi_lane(g, c.ring, c.ring.xy >= 0);
    Ln.ph = psi_lane(g, c.hc, c.hc.xy >= 0);
    Ln.ysl = c.own.sy >= 0;
    fill_coef_tile<TY, CZ>(g, ct, c.i0, c.j0, k0, c.tid, TX * TY);
    __syncthreads();   // the prologue's E-half terms read the coefficient tile
    // the tile's class: the slabs that the cells it reads PML auxiliaries of reach
    // (own, ring and halo columns, planes k0-1 .. k0+CZ; uniform over the block)
    switch (slab_class(g, c.i0 - 1, c.i0 + TX, c.j0 - 1, c.j0 + TY, k0 - 1, k0 + CZ)) {
        case 0: adj_tile<TY, CZ, 0>(g, b, Ln, c, sG, sGH, ct, k0, k1); break;
        case 1: adj_tile<TY, CZ, 1>(g, b, Ln, c, sG, sGH, ct, k0, k1); break;
        case 2: adj_tile<TY, CZ, 2>(g, b, Ln, c, sG, sGH, ct, k0, k1); break;
        case 3: adj_tile<TY, CZ, 3>(g, b, Ln, c, sG, sGH, ct, k0, k1); break;
        case 4: adj_tile<TY, CZ, 4>(g, b, Ln, c, sG, sGH, ct, k0, k1); break;
        case 5: adj_tile<TY, CZ, 5>(g, b, Ln, c, sG, sGH, ct, k0, k1); break;
        case 6: adj_tile<TY, CZ, 6>(g, b, Ln, c, sG, sGH, ct, k0, k1); break;
        default: adj_tile<TY, CZ, 7>(g, b, Ln, c, sG, sGH, ct, k0, k1); break;
    }
}

// --------------------------------------------------------------------------
// primal reversal over the interior and its shell
// --------------------------------------------------------------------------

struct Box {            // the region prim_rev sweeps: I plus a one-cell shell
    int o[3];           // origin
    int n[3];           // extent
    int tx0;            // x origin of the tiles: o[0] rounded down to a 128-byte line
    int xrow;           // x-face shell cells at position y - P of row 0 (ShellJob.xrow)
};

struct RevBufs {
    rsrc_t F0, F1, eps, src, msrc;   // primal fields in / out (E then H), source profiles
};

// What the primal reversal reads for plane k, loaded one plane ahead: H^{n+1/2}
// at plane k+1 (own cell and LDS-ring position), and E^{n+1}, eps and the source
// profile at plane k+1 (own cell and the extra +x / +y position).
struct RevIn {
    float h[3], rh[3], e[3], xe[3], ep, xep, sp, xsp;   // e, xe: E^{n+1}, or E^n on the high-face shell
    float mp;                 // magnetic-current profile of the own cell at plane k (0 off the sheet)
};

// Loop-invariant per-lane byte offsets: H of the own column and ring position
// (boundary rule), eps of the own and extra positions where they are interior in x
// and y (e, xe: also the E loads of the z face plane nz-P, whose x-y interior is
// shell), the E loads of interior planes (es, xes: interior in x and y, or on the
// x or y high face), the source box column of both, and the own cell's stores.
struct RevLanes {
    uint32_t h, r, e, xe, es, xes, src, xsrc, st, m;
};

template <int TY>
struct RevCtx {
    int i0, j0, lane, row, x, y, N, plane;
    bool live;
    Col own, ring, xcol;
    int rlx, rly, pex, pey;
};

__device__ inline bool xy_interior(const Grid& g, const Col& c) {
    return c.xy >= 0 && c.x >= g.P && c.x < g.nx - g.P && c.y >= g.P && c.y < g.ny - g.P;
}
__device__ inline uint32_t src_lane(const Grid& g, const Col& c) {
    const bool in = c.xy >= 0 && c.x >= g.src_lo[0] && c.x < g.src_hi[0] && c.y >= g.src_lo[1] && c.y < g.src_hi[1];
    return lane_off(in, (c.x - g.src_lo[0]) + (g.src_hi[0] - g.src_lo[0]) * (c.y - g.src_lo[1]));
}
// uniform byte offset of plane z in the source profile, and whether z crosses the source box
__device__ inline bool src_z(const Grid& g, int z, uint32_t& s) {
    const bool in = z >= g.src_lo[2] && z < g.src_hi[2];
    s = uni(in ? (uint32_t)((z - g.src_lo[2]) * (g.src_hi[0] - g.src_lo[0]) * (g.src_hi[1] - g.src_lo[1])) << 2 : 0u);
    return in;
}
__device__ inline bool z_interior(const Grid& g, int z) { return z >= g.P && z < g.nz - g.P; }

template <int TY, bool MS>
__device__ __forceinline__ void load_rev_in(const Grid& g, const RevBufs& b, const RevLanes& L, const RevCtx<TY>& c,
                                            int k, RevIn& d) {
    const uint32_t nb = (uint32_t)c.N << 2;
    const int z1 = bound(k + 1, g.nz, g.periodic);
    const uint32_t s1 = uni(z1 < 0 ? 0u : (uint32_t)(z1 * c.plane) << 2);
    bld3v(b.F0, z1 < 0 ? OOB : L.h, s1 + 3 * nb, nb, d.h);
    bld3v(b.F0, z1 < 0 ? OOB : L.r, s1 + 3 * nb, nb, d.rh);
    const bool zi = z1 >= 0 && z_interior(g, z1);
    const bool zh = z1 >= 0 && g.P > 0 && z1 == g.nz - g.P;    // the z high face: shell
    bld3v(b.F0, zi ? L.es : (zh ? L.e : OOB), s1, nb, d.e);
    bld3v(b.F0, zi ? L.xes : (zh ? L.xe : OOB), s1, nb, d.xe);
    const float ep = bldv(b.eps, zi ? L.e : OOB, s1), xep = bldv(b.eps, zi ? L.xe : OOB, s1);
    d.ep = ep == 0.0f ? 1.0f : ep;      // positions that are not interior read 0
    d.xep = xep == 0.0f ? 1.0f : xep;
    uint32_t ss = 0;
    const bool sz = z1 >= 0 && src_z(g, z1, ss);
    d.sp = bldv(b.src, sz ? L.src : OOB, ss);
    d.xsp = bldv(b.src, sz ? L.xsrc : OOB, ss);
    if constexpr (MS) {   // a magnetic-current sheet exists (a separate instantiation)
        uint32_t ms;
        const bool mz = box_plane(g.msrc_lo, g.msrc_hi, k, ms);
        d.mp = bldv(b.msrc, mz ? L.m : OOB, ms);
    } else {
        d.mp = 0.0f;
    }
}

// E^n at one position of plane z (column col, wrapped; extended-plane coordinates
// (ex, ey) of the LDS H planes at z (hc) and z-1 (hp)).  Interior cells are
// reversed, E^n = E^{n+1} - (dt/eps)(curl H - J); on high-face shell cells e1 is the
// recorded E^n already, and anything else reads 0.  u returns curl H - J (interior cells).
template <int TY>
__device__ __forceinline__ void e_rev(const Grid& g, const float (*hc)[TY + 2][EXT], const float (*hp)[TY + 2][EXT],
                                      int ex, int ey, const Col& col, int z, const float e1[3], float ep, float sp,
                                      float wave, float e[3], float u[3], bool& interior) {
    const int P = g.P, x = col.x, y = col.y;
    const bool inside = col.xy >= 0 && z >= 0;
    const bool iI = x >= P && x < g.nx - P, jI = y >= P && y < g.ny - P, kI = z >= P && z < g.nz - P;
    interior = inside && iI && jI && kI;
    const float hx = hc[0][ey][ex], hy = hc[1][ey][ex], hz = hc[2][ey][ex];
    u[0] = (hz - hc[2][ey - 1][ex]) - (hy - hp[1][ey][ex]);
    u[1] = (hx - hp[0][ey][ex]) - (hz - hc[2][ey][ex - 1]);
    u[2] = (hy - hc[1][ey][ex - 1]) - (hx - hc[0][ey - 1][ex]);
    const float jv = wave * sp;   // 0 outside the source box
    u[0] -= g.src_comp == 0 ? jv : 0.0f;
    u[1] -= g.src_comp == 1 ? jv : 0.0f;
    u[2] -= g.src_comp == 2 ? jv : 0.0f;
    const float cc = dt_over_eps(g.dt, ep);
    e[0] = interior ? e1[0] - cc * u[0] : e1[0];
    e[1] = interior ? e1[1] - cc * u[1] : e1[1];
    e[2] = interior ? e1[2] - cc * u[2] : e1[2];
}

// E^n of plane z on the own cell (written by its owner, with gradient and seed) and the
// extra position, into the LDS plane sE.
template <int TY>
__device__ __forceinline__ void e_plane(const Grid& g, const RevBufs& b, const RevLanes& L, const RevCtx<TY>& c,
                                        float (*sE)[TY + 1][TX + 1], const float (*hc)[TY + 2][EXT],
                                        const float (*hp)[TY + 2][EXT], int z, bool owned, const float e1[3], float ep,
                                        float sp, const float xe1[3], float xep, float xsp, float wave,
                                        float* __restrict__ Eb0, double* __restrict__ grad) {
    const int lane = c.lane, row = c.row;
    float e[3], u[3];
    bool interior;
    e_rev<TY>(g, hc, hp, lane + 1, row + 1, c.own, z, e1, ep, sp, wave, e, u, interior);
    sE[0][row][lane] = e[0];
    sE[1][row][lane] = e[1];
    sE[2][row][lane] = e[2];
    // own interior cell: store (its lane offset is OOB unless live and interior in x and y)
    const bool zst = owned && z >= 0 && z_interior(g, z);
    const uint32_t nb = (uint32_t)c.N << 2;
    bst3v(b.F1, zst ? L.st : OOB, uni(zst ? (uint32_t)(z * c.plane) << 2 : 0u), nb, e);
    if (owned && c.live && interior) {
        const float h[3] = {hc[0][row + 1][lane + 1], hc[1][row + 1][lane + 1], hc[2][row + 1][lane + 1]};
        grad_and_seed(g, Eb0, grad, c.own.x, c.own.y, z, c.own.xy + z * c.plane, e1, h, ep, u);
    }
    if (c.pex >= 0) {
        e_rev<TY>(g, hc, hp, c.pex + 1, c.pey + 1, c.xcol, z, xe1, xep, xsp, wave, e, u, interior);
        sE[0][c.pey][c.pex] = e[0];
        sE[1][c.pey][c.pex] = e[1];
        sE[2][c.pey][c.pex] = e[2];
    }
}

// The z-march of one primal-reversal tile over planes [k0, k1).  (Tiles specialised by
// what they need, as the forward and adjoint sweeps are, measured slower here: a launch
// of this sweep is about one round of the chip, so blocks of every class run side by
// side and their code paths evict each other from the instruction cache.)
template <int TY, int CZ, bool MS>
__device__ __forceinline__ void rev_tile(const Grid& g, const RevBufs& b, const RevLanes& Ln, const RevCtx<TY>& c,
                                         float (*sH)[3][TY + 2][EXT], float (*sE)[3][TY + 1][TX + 1], int k0, int k1,
                                         float wave, float mwave, float* __restrict__ Eb0, double* __restrict__ grad) {
    const int lane = c.lane, row = c.row, P = g.P;
    const uint32_t nb = (uint32_t)c.N << 2;
    const float dt = g.dt;
    // prologue: H^{n+1/2} planes k0-1 and k0 into LDS, then E^n at k0
    RevIn pin[2];
    {
        const int zm = bound(k0 - 1, g.nz, g.periodic), z0 = bound(k0, g.nz, g.periodic);
        const uint32_t sm = uni(zm < 0 ? 0u : (uint32_t)(zm * c.plane) << 2), s0 = uni((uint32_t)(z0 * c.plane) << 2);
        float hm[3], rhm[3], h0[3], rh0[3], e1[3], xe1[3];
        bld3v(b.F0, zm < 0 ? OOB : Ln.h, sm + 3 * nb, nb, hm);
        bld3v(b.F0, zm < 0 ? OOB : Ln.r, sm + 3 * nb, nb, rhm);
        bld3v(b.F0, Ln.h, s0 + 3 * nb, nb, h0);
        bld3v(b.F0, Ln.r, s0 + 3 * nb, nb, rh0);
        const bool zi = z_interior(g, z0), zh = P > 0 && z0 == g.nz - P;
        bld3v(b.F0, zi ? Ln.es : (zh ? Ln.e : OOB), s0, nb, e1);
        bld3v(b.F0, zi ? Ln.xes : (zh ? Ln.xe : OOB), s0, nb, xe1);
        float ep = bldv(b.eps, zi ? Ln.e : OOB, s0), xep = bldv(b.eps, zi ? Ln.xe : OOB, s0);
        uint32_t ss;
        const bool sz = src_z(g, z0, ss);
        const float sp = bldv(b.src, sz ? Ln.src : OOB, ss), xsp = bldv(b.src, sz ? Ln.xsrc : OOB, ss);
        load_rev_in<TY, MS>(g, b, Ln, c, k0, pin[0]);
        ep = ep == 0.0f ? 1.0f : ep;
        xep = xep == 0.0f ? 1.0f : xep;
        #pragma unroll
        for (int q = 0; q < 3; ++q) {
            sH[0][q][row + 1][lane + 1] = hm[q];
            sH[1][q][row + 1][lane + 1] = h0[q];
        }
        if (c.rlx >= 0) {
            #pragma unroll
            for (int q = 0; q < 3; ++q) { sH[0][q][c.rly][c.rlx] = rhm[q]; sH[1][q][c.rly][c.rlx] = rh0[q]; }
        }
        __syncthreads();
        e_plane<TY>(g, b, Ln, c, sE[0], sH[1], sH[0], z0, true, e1, ep, sp, xe1, xep, xsp, wave, Eb0, grad);
    }
    __syncthreads();   // the first plane overwrites sH[0], which the prologue has just read
    #pragma unroll
    for (int kk = 0; kk < CZ; ++kk) {
        const int k = k0 + kk;
        if (kk + 1 < CZ) load_rev_in<TY, MS>(g, b, Ln, c, min(k + 1, g.nz - 1), pin[(kk + 1) & 1]);
        if (k >= k1) continue;
        const int hc = (kk + 1) & 1, hn = 1 - hc;      // H plane k in sH[hc]
        const int ec = kk & 1, en = 1 - ec;            // E^n plane k in sE[ec]
        const RevIn& in = pin[kk & 1];
        #pragma unroll
        for (int q = 0; q < 3; ++q) sH[hn][q][row + 1][lane + 1] = in.h[q];
        if (c.rlx >= 0) {
            #pragma unroll
            for (int q = 0; q < 3; ++q) sH[hn][q][c.rly][c.rlx] = in.rh[q];
        }
        __syncthreads();
        // E^n at plane k+1 (own cell, and the +x column / +y row)
        const int z1 = bound(k + 1, g.nz, g.periodic);
        e_plane<TY>(g, b, Ln, c, sE[en], sH[hn], sH[hc], z1, k + 1 < k1, in.e, in.ep, in.sp, in.xe, in.xep, in.xsp,
                    wave, Eb0, grad);
        __syncthreads();
        // H^{n-1/2} at plane k on the tile (interior cells; lane offset OOB elsewhere)
        const bool kI = z_interior(g, k);
        float h[3];
        {
            const float exc = sE[ec][0][row][lane], eyc = sE[ec][1][row][lane], ezc = sE[ec][2][row][lane];
            h[0] = sH[hc][0][row + 1][lane + 1] + dt * ((sE[ec][2][row + 1][lane] - ezc) - (sE[en][1][row][lane] - eyc));
            h[1] = sH[hc][1][row + 1][lane + 1] + dt * ((sE[en][0][row][lane] - exc) - (sE[ec][2][row][lane + 1] - ezc));
            h[2] = sH[hc][2][row + 1][lane + 1] + dt * ((sE[ec][1][row][lane + 1] - eyc) - (sE[ec][0][row + 1][lane] - exc));
            const float m = MS ? dt * mwave * in.mp : 0.0f;   // the step's magnetic current, 0 off its sheet
            h[0] += g.msrc_comp == 0 ? m : 0.0f;
            h[1] += g.msrc_comp == 1 ? m : 0.0f;
            h[2] += g.msrc_comp == 2 ? m : 0.0f;
        }
        bst3v(b.F1, kI ? Ln.st : OOB, uni(((uint32_t)(k * c.plane) << 2) + 3 * nb), nb, h);
    }
}

// One reverse primal step over the box: (E^{n+1}, H^{n+1/2}) in F0 -> (E^n, H^{n-1/2})
// in F1 on the interior, with the gradient and the loss seed.  The interface shell of
// the step (E^n on the high faces, in F0; H^{n-1/2} on the low faces, in F1) is
// written beforehand from the store (by the previous adjoint launch, or
// k_inject_shell on the first reverse step); the sweep reads the E part of it.
#ifndef FDTD_REV_WAVES
#define FDTD_REV_WAVES 1
#endif
template <int TY, int CZ, bool MS>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(FDTD_REV_WAVES))) void k_prim_rev(
    Grid g, Tiling tl, Box bx, const float* __restrict__ F0, float* __restrict__ F1, const float* __restrict__ eps,
    float* __restrict__ Eb0, float wave, float mwave, double* __restrict__ grad) {
    __shared__ float sH[2][3][TY + 2][EXT];       // H^{n+1/2}, extended planes
    __shared__ float sE[2][3][TY + 1][TX + 1];     // E^n on the tile plus the +x column / +y row
    const int L = logical_tile(tl);
    const int tix = L % tl.ntx, tiy = (L / tl.ntx) % tl.nty, tiz = L / (tl.ntx * tl.nty);
    RevCtx<TY> c;
    c.i0 = bx.tx0 + tix * TX;
    c.j0 = bx.o[1] + tiy * TY;
    const int k0 = bx.o[2] + tiz * CZ;
    const int k1 = min(k0 + CZ, bx.o[2] + bx.n[2]);
    c.lane = threadIdx.x;
    c.row = threadIdx.y;
    const int lane = c.lane, row = c.row;
    c.x = c.i0 + lane;
    c.y = c.j0 + row;
    c.live = c.x >= bx.o[0] && c.x < bx.o[0] + bx.n[0] && c.y < bx.o[1] + bx.n[1];
    c.N = (int)g.N;
    c.plane = g.nx * g.ny;
    const int N = c.N, P = g.P;
    RevBufs b;
    b.F0 = make_rsrc(F0, (uint32_t)(6 * N) * 4u);
    b.F1 = make_rsrc(F1, (uint32_t)(6 * N) * 4u);
    b.eps = make_rsrc(eps, (uint32_t)(c.plane * g.nz) * 4u);
    b.src = make_rsrc(g.src_profile, (uint32_t)((g.src_hi[0] - g.src_lo[0]) * (g.src_hi[1] - g.src_lo[1]) *
                                                (g.src_hi[2] - g.src_lo[2])) * 4u);
    if constexpr (MS)
        b.msrc = make_rsrc(g.msrc_profile, (uint32_t)((g.msrc_hi[0] - g.msrc_lo[0]) * (g.msrc_hi[1] - g.msrc_lo[1]) *
                                                      (g.msrc_hi[2] - g.msrc_lo[2])) * 4u);
    c.own = make_col(g, c.x, c.y);
    c.rlx = c.rly = -1;
    c.ring.xy = -1;
    c.ring.x = c.ring.y = -1;
    if (row == 0) { c.rlx = lane + 1; c.rly = 0; c.ring = make_col(g, c.i0 + lane, c.j0 - 1); }
    else if (row == 1) { c.rlx = lane + 1; c.rly = TY + 1; c.ring = make_col(g, c.i0 + lane, c.j0 + TY); }
    else if (row == 2 && lane < TY + 2) { c.rlx = 0; c.rly = lane; c.ring = make_col(g, c.i0 - 1, c.j0 - 1 + lane); }
    else if (row == 3 && lane < TY + 2) { c.rlx = EXT - 1; c.rly = lane; c.ring = make_col(g, c.i0 + TX, c.j0 - 1 + lane); }
    // extra E^n positions: the row y = j0+TY (wave 2) and the column x = i0+TX (wave 3),
    // away from the ring rows of waves 0 and 1
    c.pex = c.pey = -1;
    c.xcol.xy = -1;
    c.xcol.x = c.xcol.y = -1;
    if (row == 2) { c.pex = lane; c.pey = TY; }
    else if (row == 3 && lane < TY + 1) { c.pex = TX; c.pey = lane; }
    if (c.pex >= 0) c.xcol = make_col(g, c.i0 + c.pex, c.j0 + c.pey);
    RevLanes Ln;
    // without wrap-around, idle lanes (outside the box) are never a neighbour of a box cell
    // H of a column on the low x face (its interior rows) comes from row 0 with xrow
    auto hface = [&](const Col& q) {
        return bx.xrow && q.x == P - 1 && q.y >= P && q.y < g.ny - P ? q.y - P : q.xy;
    };
    Ln.h = lane_off(c.own.xy >= 0 && (c.live || g.periodic), hface(c.own));
    Ln.r = lane_off(c.ring.xy >= 0, hface(c.ring));
    Ln.e = lane_off(xy_interior(g, c.own), c.own.xy);
    Ln.xe = lane_off(xy_interior(g, c.xcol), c.xcol.xy);
    Ln.src = src_lane(g, c.own);
    Ln.xsrc = src_lane(g, c.xcol);
    Ln.st = lane_off(c.live && xy_interior(g, c.own), c.own.xy);
    Ln.m = box_lane(g.msrc_lo, g.msrc_hi, c.own);
    {
        // interior in x and y, or on the x or y high face (the E^n shell in the input buffer)
        auto es = [&](const Col& q) {
            const bool iI = q.x >= P && q.x < g.nx - P, jI = q.y >= P && q.y < g.ny - P;
            const bool xface = P > 0 && q.x == g.nx - P && jI;
            const bool face = xface || (P > 0 && q.y == g.ny - P && iI);
            return lane_off(q.xy >= 0 && (xy_interior(g, q) || face), bx.xrow && xface ? q.y - P : q.xy);
        };
        Ln.es = es(c.own);
        Ln.xes = es(c.xcol);
    }

    rev_tile<TY, CZ, MS>(g, b, Ln, c, sH, sE, k0, k1, wave, mwave, Eb0, grad);
}

__global__ void k_scale_grad(double* g, long long n, const double* s) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[i] *= *s;
}

static long long shell_thread_count(const Grid& g) {
    return 2 * ((long long)g.my * g.mz + (long long)g.mx * g.mz + (long long)g.mx * g.my);
}

template <int TY, int CZ>
static void launch_adj_t(const Grid& g, const Tiling& t, const float* A0, float* A1, const float* eps, float* psi,
                         int pcopy, const ShellJob* job, hipStream_t s) {
    ShellJob j{};
    long long extra = 0;
    if (job && g.P > 0 && (job->do_e || job->do_h)) {
        j = *job;
        extra = (shell_thread_count(g) + TX * TY - 1) / (TX * TY);
    }
    launch_kernel(K_ADJ_STEP, k_adj_step<TY, CZ>, dim3((unsigned)(t.count + extra)), dim3(TX, TY), s, g, t, A0, A1,
                  eps, psi, pcopy, j);
}

void launch_adj_step(const Grid& g, const Tiling& t, const float* A0, float* A1, const float* eps, float* psi,
                     int pcopy, const ShellJob* job, hipStream_t s) {
    if (t.ty == 4 && t.cz == 4) launch_adj_t<4, 4>(g, t, A0, A1, eps, psi, pcopy, job, s);
    else if (t.ty == 4) launch_adj_t<4, 8>(g, t, A0, A1, eps, psi, pcopy, job, s);
    else if (t.cz == 4) launch_adj_t<8, 4>(g, t, A0, A1, eps, psi, pcopy, job, s);
    else launch_adj_t<8, 8>(g, t, A0, A1, eps, psi, pcopy, job, s);
}

template <int TY, int CZ>
static void launch_prim_rev_t(const Grid& g, const Tiling& t, const Box& b, const float* F0, float* F1,
                              const float* eps, float* Eb0, float wave, float mwave, double* grad, hipStream_t s) {
    if (g.msrc_hi[0] > g.msrc_lo[0])
        launch_kernel(K_PRIM_REV, k_prim_rev<TY, CZ, true>, dim3(t.count), dim3(TX, TY), s, g, t, b, F0, F1, eps, Eb0,
                      wave, mwave, grad);
    else
        launch_kernel(K_PRIM_REV, k_prim_rev<TY, CZ, false>, dim3(t.count), dim3(TX, TY), s, g, t, b, F0, F1, eps,
                      Eb0, wave, mwave, grad);
}

void launch_prim_rev(const Grid& g, const Tiling& t, const int box_o[3], const int box_n[3], int tile_x0, int xrow,
                     const float* F0, float* F1, const float* eps, float* Eb0, float wave, float mwave, double* grad,
                     hipStream_t s) {
    Box b;
    for (int d = 0; d < 3; ++d) { b.o[d] = box_o[d]; b.n[d] = box_n[d]; }
    b.tx0 = tile_x0;
    b.xrow = xrow;
    if (t.ty == 4 && t.cz == 4) launch_prim_rev_t<4, 4>(g, t, b, F0, F1, eps, Eb0, wave, mwave, grad, s);
    else if (t.ty == 4 && t.cz == 5) launch_prim_rev_t<4, 5>(g, t, b, F0, F1, eps, Eb0, wave, mwave, grad, s);
    else if (t.ty == 4 && t.cz == 6) launch_prim_rev_t<4, 6>(g, t, b, F0, F1, eps, Eb0, wave, mwave, grad, s);
    else if (t.ty == 4) launch_prim_rev_t<4, 8>(g, t, b, F0, F1, eps, Eb0, wave, mwave, grad, s);
    else if (t.cz == 4) launch_prim_rev_t<8, 4>(g, t, b, F0, F1, eps, Eb0, wave, mwave, grad, s);
    else launch_prim_rev_t<8, 8>(g, t, b, F0, F1, eps, Eb0, wave, mwave, grad, s);
}

void launch_inject_shell(const Grid& g, const ShellJob& job, hipStream_t s) {
    if (g.P == 0 || (!job.do_e && !job.do_h)) return;
    const long long n = shell_thread_count(g);
    with_dtype(g.dtype, [&]<int DT>() {
        launch_kernel(K_INJECT, k_inject_shell<DT>, dim3((unsigned)((n + 255) / 256)), dim3(256), s, g, job);
    });
}

void launch_scale_grad(double* grad, long long n, const double* scale, hipStream_t s) {
    if (n <= 0) return;
    launch_kernel(K_SCALE_GRAD, k_scale_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), s, grad, n, scale);
}

}  // namespace fdtd
