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
#include "march.h"

namespace fdtd {

// --------------------------------------------------------------------------
// adjoint sweep
// --------------------------------------------------------------------------

// gbar of the six E-half terms at (x, y, z) from v = (dt/eps) Ebar_eff.
// Terms: 0 (vx,+,y) 1 (vx,-,z) 2 (vy,+,z) 3 (vy,-,x) 4 (vz,+,x) 5 (vz,-,y).
__device__ inline void gbar_e(const Grid& g, int x, int y, int z, float vx, float vy, float vz,
                              const float* __restrict__ psi_in, float* __restrict__ psi_out, float o[6]) {
    o[0] = vx; o[1] = -vx; o[2] = vy; o[3] = -vy; o[4] = vz; o[5] = -vz;
    const int P = g.P;
    if (P == 0) return;
    const float* b = g.coef;
    const float* a = g.coef + 2 * P;
    const float* kv = g.coef + 4 * P;
    int s = slab_coord(x, g.nx, P);
    if (s >= 0) {
        const int sl = (int)g.slab[0];
        const int q = (int)(g.psi_off[0] + 2 * g.slab[0]) + s + 2 * P * (y + g.ny * z);
        const float pa = psi_in[q] + o[3], pb = psi_in[q + sl] + o[4];
        o[3] = kv[s] * o[3] + a[s] * pa;
        o[4] = kv[s] * o[4] + a[s] * pb;
        if (psi_out) { psi_out[q] = b[s] * pa; psi_out[q + sl] = b[s] * pb; }
    }
    s = slab_coord(y, g.ny, P);
    if (s >= 0) {
        const int sl = (int)g.slab[1];
        const int q = (int)(g.psi_off[1] + 2 * g.slab[1]) + x + g.nx * (s + 2 * P * z);
        const float pa = psi_in[q] + o[0], pb = psi_in[q + sl] + o[5];
        o[0] = kv[s] * o[0] + a[s] * pa;
        o[5] = kv[s] * o[5] + a[s] * pb;
        if (psi_out) { psi_out[q] = b[s] * pa; psi_out[q + sl] = b[s] * pb; }
    }
    s = slab_coord(z, g.nz, P);
    if (s >= 0) {
        const int sl = (int)g.slab[2];
        const int q = (int)(g.psi_off[2] + 2 * g.slab[2]) + x + g.nx * (y + g.ny * s);
        const float pa = psi_in[q] + o[1], pb = psi_in[q + sl] + o[2];
        o[1] = kv[s] * o[1] + a[s] * pa;
        o[2] = kv[s] * o[2] + a[s] * pb;
        if (psi_out) { psi_out[q] = b[s] * pa; psi_out[q + sl] = b[s] * pb; }
    }
}

// gbar of the six H-half terms at (x, y, z) from w = -dt Hbar_new.
// Terms: 0 (wx,+,y) 1 (wx,-,z) 2 (wy,+,z) 3 (wy,-,x) 4 (wz,+,x) 5 (wz,-,y).
__device__ inline void gbar_h(const Grid& g, int x, int y, int z, float wx, float wy, float wz,
                              const float* __restrict__ psi_in, float* __restrict__ psi_out, float o[6]) {
    o[0] = wx; o[1] = -wx; o[2] = wy; o[3] = -wy; o[4] = wz; o[5] = -wz;
    const int P = g.P;
    if (P == 0) return;
    const float* b = g.coef + 6 * P;
    const float* a = g.coef + 8 * P;
    const float* kv = g.coef + 10 * P;
    int s = slab_coord(x, g.nx, P);
    if (s >= 0) {
        const int sl = (int)g.slab[0];
        const int q = (int)g.psi_off[0] + s + 2 * P * (y + g.ny * z);
        const float pa = psi_in[q] + o[3], pb = psi_in[q + sl] + o[4];
        o[3] = kv[s] * o[3] + a[s] * pa;
        o[4] = kv[s] * o[4] + a[s] * pb;
        if (psi_out) { psi_out[q] = b[s] * pa; psi_out[q + sl] = b[s] * pb; }
    }
    s = slab_coord(y, g.ny, P);
    if (s >= 0) {
        const int sl = (int)g.slab[1];
        const int q = (int)g.psi_off[1] + x + g.nx * (s + 2 * P * z);
        const float pa = psi_in[q] + o[0], pb = psi_in[q + sl] + o[5];
        o[0] = kv[s] * o[0] + a[s] * pa;
        o[5] = kv[s] * o[5] + a[s] * pb;
        if (psi_out) { psi_out[q] = b[s] * pa; psi_out[q + sl] = b[s] * pb; }
    }
    s = slab_coord(z, g.nz, P);
    if (s >= 0) {
        const int sl = (int)g.slab[2];
        const int q = (int)g.psi_off[2] + x + g.nx * (y + g.ny * s);
        const float pa = psi_in[q] + o[1], pb = psi_in[q + sl] + o[2];
        o[1] = kv[s] * o[1] + a[s] * pa;
        o[2] = kv[s] * o[2] + a[s] * pb;
        if (psi_out) { psi_out[q] = b[s] * pa; psi_out[q + sl] = b[s] * pb; }
    }
}

// E-half gbar of one extended-plane position (ex, ey) at plane z into sG[t][ey][ex];
// returns Ebar_eff there.  Positions outside the domain (zero boundary) give 0.
template <int TY>
__device__ inline void ge_position(const Grid& g, float (*sG)[TY + 2][EXT], int ex, int ey, int xr, int yr, int z,
                                   const float* __restrict__ Eb0, const float* __restrict__ Es,
                                   const float* __restrict__ eps, const float* __restrict__ psi_in,
                                   float* __restrict__ psi_out, float eb[3]) {
    const int x = bound(xr, g.nx, g.periodic), y = bound(yr, g.ny, g.periodic), zb = bound(z, g.nz, g.periodic);
    float o[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    eb[0] = eb[1] = eb[2] = 0.0f;
    if ((x | y | zb) >= 0) {
        const int N = (int)g.N;
        const int idx = x + g.nx * (y + g.ny * zb);
        eb[0] = Eb0[idx];
        eb[1] = Eb0[N + idx];
        eb[2] = Eb0[2 * N + idx];
        if (in_box(x, y, zb, g.det_lo, g.det_hi)) {       // this step's loss seed 2 E^{n+1}
            eb[0] += 2.0f * Es[idx];
            eb[1] += 2.0f * Es[N + idx];
            eb[2] += 2.0f * Es[2 * N + idx];
        }
        const float c = g.dt / eps[idx];
        gbar_e(g, x, y, zb, c * eb[0], c * eb[1], c * eb[2], psi_in, psi_out, o);
    }
    #pragma unroll
    for (int t = 0; t < 6; ++t) sG[t][ey][ex] = o[t];
}

// E-half gbar on the extended plane z (tile plus a one-cell ring); the owner
// of a tile cell writes its PML auxiliaries when `owned`.  Returns the own
// cell's Ebar_eff.
template <int TY>
__device__ inline void ge_plane(const Grid& g, float (*sG)[TY + 2][EXT], int i0, int j0, int z, bool owned,
                                const float* Eb0, const float* Es, const float* eps, const float* psi_in,
                                float* psi_out, float eb[3]) {
    const int lane = threadIdx.x, ty = threadIdx.y;
    const bool live = i0 + lane < g.nx && j0 + ty < g.ny;
    ge_position<TY>(g, sG, lane + 1, ty + 1, i0 + lane, j0 + ty, z, Eb0, Es, eps, psi_in,
                    (owned && live) ? psi_out : nullptr, eb);
    float dummy[3];
    if (ty == 0)
        ge_position<TY>(g, sG, lane + 1, 0, i0 + lane, j0 - 1, z, Eb0, Es, eps, psi_in, nullptr, dummy);
    else if (ty == 1)
        ge_position<TY>(g, sG, lane + 1, TY + 1, i0 + lane, j0 + TY, z, Eb0, Es, eps, psi_in, nullptr, dummy);
    else if (ty == 2 && lane < TY + 2)
        ge_position<TY>(g, sG, 0, lane, i0 - 1, j0 - 1 + lane, z, Eb0, Es, eps, psi_in, nullptr, dummy);
    else if (ty == 3 && lane < TY + 2)
        ge_position<TY>(g, sG, EXT - 1, lane, i0 + TX, j0 - 1 + lane, z, Eb0, Es, eps, psi_in, nullptr, dummy);
}

// Hbar after the E-half transpose at the cell of extended coordinates (ex, ey):
// Hbar0 + sum_t (gbar_t(p) - gbar_t(p + e_d)), +z from the next plane.
template <int TY>
__device__ inline void hbar_new(const float (*cur)[TY + 2][EXT], const float (*nxt)[TY + 2][EXT], int ex, int ey,
                                float h0x, float h0y, float h0z, float& hx, float& hy, float& hz) {
    hx = h0x + (cur[2][ey][ex] - nxt[2][ey][ex]) + (cur[5][ey][ex] - cur[5][ey + 1][ex]);
    hy = h0y + (cur[1][ey][ex] - nxt[1][ey][ex]) + (cur[4][ey][ex] - cur[4][ey][ex + 1]);
    hz = h0z + (cur[0][ey][ex] - cur[0][ey + 1][ex]) + (cur[3][ey][ex] - cur[3][ey][ex + 1]);
}

template <int TY>
__global__ __launch_bounds__(TX * TY) void k_adj_step(Grid g, Tiling tl, const float* __restrict__ Eb0,
                                                      const float* __restrict__ Hb0, float* __restrict__ Eb1,
                                                      float* __restrict__ Hb1, const float* __restrict__ Es,
                                                      const float* __restrict__ eps, const float* __restrict__ psi_in,
                                                      float* __restrict__ psi_out) {
    __shared__ float sG[2][6][TY + 2][EXT];
    __shared__ float sGH[6][TY + 1][TX + 1];
    const int L = logical_tile(tl.count);
    const int tix = L % tl.ntx, tiy = (L / tl.ntx) % tl.nty, tiz = L / (tl.ntx * tl.nty);
    const int i0 = tix * TX, j0 = tiy * TY, k0 = tiz * tl.cz;
    const int k1 = min(k0 + tl.cz, g.nz);
    const int lane = threadIdx.x, row = threadIdx.y;
    const int tid = row * TX + lane;
    const int x = i0 + lane, y = j0 + row;
    const bool live = x < g.nx && y < g.ny;
    const int N = (int)g.N;
    const float dt = g.dt;

    // halo cell of the first half (as in the forward step): row y = j0-1 or column x = i0-1
    int hex = -1, hey = -1, hxg = -1, hyg = -1;
    if (tid < TX + TY) {
        if (tid < TX) { hex = tid + 1; hey = 0; } else { hex = 0; hey = tid - TX + 1; }
        const int xr = i0 - 1 + hex, yr = j0 - 1 + hey;
        if (xr < g.nx && yr < g.ny) {
            hxg = bound(xr, g.nx, g.periodic);
            hyg = bound(yr, g.ny, g.periodic);
        }
    }

    float ebc[3], ebn[3];
    ge_plane<TY>(g, sG[0], i0, j0, k0 - 1, false, Eb0, Es, eps, psi_in, psi_out, ebn);
    ge_plane<TY>(g, sG[1], i0, j0, k0, true, Eb0, Es, eps, psi_in, psi_out, ebc);
    __syncthreads();
    // H-half gbar of this column at k0 - 1 (terms along z), from Hbar after the E half there
    float g1p = 0.0f, g2p = 0.0f;
    {
        const int zb = bound(k0 - 1, g.nz, g.periodic);
        if (live && zb >= 0) {
            const int idx = x + g.nx * (y + g.ny * zb);
            float hx, hy, hz, o[6];
            hbar_new<TY>(sG[0], sG[1], lane + 1, row + 1, Hb0[idx], Hb0[N + idx], Hb0[2 * N + idx], hx, hy, hz);
            gbar_h(g, x, y, zb, -dt * hx, -dt * hy, -dt * hz, psi_in, nullptr, o);
            g1p = o[1];
            g2p = o[2];
        }
    }
    int cur = 1;
    for (int k = k0; k < k1; ++k) {
        const int nxt = 1 - cur;
        __syncthreads();
        ge_plane<TY>(g, sG[nxt], i0, j0, k + 1, k + 1 < k1, Eb0, Es, eps, psi_in, psi_out, ebn);
        __syncthreads();
        float og[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        #pragma unroll 1
        for (int pass = 0; pass < 2; ++pass) {
            const bool own = pass == 0;
            if (!own && hex < 0) break;
            const bool active = own ? live : (hxg >= 0 && hyg >= 0);
            const int cex = own ? lane + 1 : hex, cey = own ? row + 1 : hey;
            const int cx = own ? x : hxg, cy = own ? y : hyg;
            float o[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (active) {
                const int idx = cx + g.nx * (cy + g.ny * k);
                float hx, hy, hz;
                hbar_new<TY>(sG[cur], sG[nxt], cex, cey, Hb0[idx], Hb0[N + idx], Hb0[2 * N + idx], hx, hy, hz);
                if (own) {
                    Hb1[idx] = hx;
                    Hb1[N + idx] = hy;
                    Hb1[2 * N + idx] = hz;
                }
                gbar_h(g, cx, cy, k, -dt * hx, -dt * hy, -dt * hz, psi_in, own ? psi_out : nullptr, o);
            }
            #pragma unroll
            for (int t = 0; t < 6; ++t) sGH[t][cey][cex] = o[t];
            if (own) {
                #pragma unroll
                for (int t = 0; t < 6; ++t) og[t] = o[t];
            }
        }
        __syncthreads();
        if (live) {
            const int idx = x + g.nx * (y + g.ny * k);
            // Ex <- terms 2 (z), 5 (y); Ey <- 1 (z), 4 (x); Ez <- 0 (y), 3 (x)
            Eb1[idx] = ebc[0] + (g2p - og[2]) + (sGH[5][row][lane + 1] - og[5]);
            Eb1[N + idx] = ebc[1] + (g1p - og[1]) + (sGH[4][row + 1][lane] - og[4]);
            Eb1[2 * N + idx] = ebc[2] + (sGH[0][row][lane + 1] - og[0]) + (sGH[3][row + 1][lane] - og[3]);
        }
        g1p = og[1];
        g2p = og[2];
        ebc[0] = ebn[0]; ebc[1] = ebn[1]; ebc[2] = ebn[2];
        cur = nxt;
    }
}

// --------------------------------------------------------------------------
// primal reversal over the interior and its shell
// --------------------------------------------------------------------------

struct Box {            // the region prim_rev sweeps: I plus a one-cell shell
    int o[3];           // origin
    int n[3];           // extent
};

// E^n at one position of plane z (global x, y) from the LDS planes of
// H^{n+1/2} at z (hc) and z - 1 (hp), extended-plane coordinates (ex, ey).
// Interior cells are reversed; high-face shell cells take the recorded values;
// anything else is unused and set to 0.  Also returns U - J for the gradient.
template <int TY>
__device__ __forceinline__ void e_rev_position(const Grid& g, const float (*hc)[TY + 2][EXT], const float (*hp)[TY + 2][EXT],
                                      int ex, int ey, int x, int y, int z, const float* __restrict__ E0,
                                      const float* __restrict__ eps, const void* __restrict__ store,
                                      const Interp& qE, float wave, float e[3], float uj[3], bool& interior) {
    const int P = g.P;
    e[0] = e[1] = e[2] = 0.0f;
    uj[0] = uj[1] = uj[2] = 0.0f;
    interior = false;
    // positions past the edge wrap (periodic grid) or are zero
    x = bound(x, g.nx, g.periodic);
    y = bound(y, g.ny, g.periodic);
    z = bound(z, g.nz, g.periodic);
    if ((x | y | z) < 0) return;
    const bool iI = x >= P && x < g.nx - P, jI = y >= P && y < g.ny - P, kI = z >= P && z < g.nz - P;
    if (iI && jI && kI) {
        interior = true;
        const int N = (int)g.N;
        const int idx = x + g.nx * (y + g.ny * z);
        const float hx = hc[0][ey][ex], hy = hc[1][ey][ex], hz = hc[2][ey][ex];
        float ux = (hz - hc[2][ey - 1][ex]) - (hy - hp[1][ey][ex]);
        float uy = (hx - hp[0][ey][ex]) - (hz - hc[2][ey][ex - 1]);
        float uz = (hy - hc[1][ey][ex - 1]) - (hx - hc[0][ey - 1][ex]);
        if (in_box(x, y, z, g.src_lo, g.src_hi)) {
            const int sxn = g.src_hi[0] - g.src_lo[0], syn = g.src_hi[1] - g.src_lo[1];
            const float jv = wave * g.src_profile[(x - g.src_lo[0]) + sxn * ((y - g.src_lo[1]) + syn * (z - g.src_lo[2]))];
            if (g.src_comp == 0) ux -= jv; else if (g.src_comp == 1) uy -= jv; else uz -= jv;
        }
        const float c = g.dt / eps[idx];
        e[0] = E0[idx] - c * ux;
        e[1] = E0[N + idx] - c * uy;
        e[2] = E0[2 * N + idx] - c * uz;
        uj[0] = ux; uj[1] = uy; uj[2] = uz;
        return;
    }
    if (P == 0) return;
    if (x == g.nx - P && jI && kI) {
        const int o = (z - P) * g.my + (y - P);
        e[1] = shell_value(g, store, qE, 6, o);
        e[2] = shell_value(g, store, qE, 7, o);
    } else if (y == g.ny - P && iI && kI) {
        const int o = (z - P) * g.mx + (x - P);
        e[2] = shell_value(g, store, qE, 8, o);
        e[0] = shell_value(g, store, qE, 9, o);
    } else if (z == g.nz - P && iI && jI) {
        const int o = (y - P) * g.mx + (x - P);
        e[0] = shell_value(g, store, qE, 10, o);
        e[1] = shell_value(g, store, qE, 11, o);
    }
}

// E^n at sE position (ex, ey) of plane z (global x = i0 + ex, y = j0 + ey) into sE[.][ey][ex];
// the owning block also writes it and accumulates the gradient there.
template <int TY>
__device__ __forceinline__ void e_pos(const Grid& g, float (*sE)[TY + 1][TX + 1], const float (*hc)[TY + 2][EXT],
                                      const float (*hp)[TY + 2][EXT], int i0, int j0, int z, int ex, int ey,
                                      bool owner, const float* __restrict__ E0, float* __restrict__ E1,
                                      const float* __restrict__ eps, const float* __restrict__ Eb0,
                                      const void* __restrict__ store, const Interp& qE, float wave,
                                      double* __restrict__ grad) {
    float e[3], uj[3];
    bool interior;
    const int xg = i0 + ex, yg = j0 + ey;
    e_rev_position<TY>(g, hc, hp, ex + 1, ey + 1, xg, yg, z, E0, eps, store, qE, wave, e, uj, interior);
    sE[0][ey][ex] = e[0];
    sE[1][ey][ex] = e[1];
    sE[2][ey][ex] = e[2];
    if (owner && interior) {
        const int N = (int)g.N;
        const int idx = xg + g.nx * (yg + g.ny * z);
        E1[idx] = e[0];
        E1[N + idx] = e[1];
        E1[2 * N + idx] = e[2];
        if (in_box(xg, yg, z, g.des_lo, g.des_hi)) {
            float ebx = Eb0[idx], eby = Eb0[N + idx], ebz = Eb0[2 * N + idx];
            if (in_box(xg, yg, z, g.det_lo, g.det_hi)) {          // this step's loss seed 2 E^{n+1}
                ebx += 2.0f * E0[idx];
                eby += 2.0f * E0[N + idx];
                ebz += 2.0f * E0[2 * N + idx];
            }
            const int dx = g.des_hi[0] - g.des_lo[0], dy = g.des_hi[1] - g.des_lo[1];
            const int di = (xg - g.des_lo[0]) + dx * ((yg - g.des_lo[1]) + dy * (z - g.des_lo[2]));
            const double ee = (double)eps[idx];
            const double s = (double)ebx * uj[0] + (double)eby * uj[1] + (double)ebz * uj[2];
            grad[di] -= (double)g.dt / (ee * ee) * s;
        }
    }
}

template <int TY>
__global__ __launch_bounds__(TX * TY) void k_prim_rev(Grid g, Tiling tl, Box bx, const float* __restrict__ E0,
                                                      const float* __restrict__ H0, float* __restrict__ E1,
                                                      float* __restrict__ H1, const float* __restrict__ eps,
                                                      const float* __restrict__ Eb0, const void* __restrict__ store,
                                                      Interp qE, Interp qH, int inject_h, float wave,
                                                      double* __restrict__ grad) {
    __shared__ float sH[2][3][TY + 2][EXT];       // H^{n+1/2}, extended planes
    __shared__ float sE[2][3][TY + 1][TX + 1];     // E^n on the tile plus the +x column / +y row
    const int L = logical_tile(tl.count);
    const int tix = L % tl.ntx, tiy = (L / tl.ntx) % tl.nty, tiz = L / (tl.ntx * tl.nty);
    const int i0 = bx.o[0] + tix * TX, j0 = bx.o[1] + tiy * TY, k0 = bx.o[2] + tiz * tl.cz;
    const int k1 = min(k0 + tl.cz, bx.o[2] + bx.n[2]);
    const int lane = threadIdx.x, row = threadIdx.y;
    const int tid = row * TX + lane;
    const int x = i0 + lane, y = j0 + row;
    const bool live = x < bx.o[0] + bx.n[0] && y < bx.o[1] + bx.n[1];
    const int N = (int)g.N;
    const int P = g.P;
    const float dt = g.dt;

    // extra E^n position of the first half: the column x = i0+TX (tid < TY+1) or the
    // row y = j0+TY (TY+1 <= tid < TY+1+TX); (ex, ey) in the sE plane
    int pex = -1, pey = -1;
    if (tid < TY + 1) { pex = TX; pey = tid; }
    else if (tid < TY + 1 + TX) { pex = tid - TY - 1; pey = TY; }

    // prologue: H^{n+1/2} planes k0-1 and k0, then E^n at k0
    load_ext_plane<TY>(sH[0], H0, N, g, i0, j0, k0 - 1);
    load_ext_plane<TY>(sH[1], H0, N, g, i0, j0, k0);
    __syncthreads();
    #pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1 && pex < 0) break;
        e_pos<TY>(g, sE[0], sH[1], sH[0], i0, j0, k0, pass ? pex : lane, pass ? pey : row, pass == 0 && live, E0, E1,
                  eps, Eb0, store, qE, wave, grad);
    }
    int hc = 1;      // slot of the H plane k in sH
    int ec = 0;      // slot of the E^n plane k in sE
    for (int k = k0; k < k1; ++k) {
        const int hn = 1 - hc, en = 1 - ec;
        __syncthreads();                                   // sH[hn] (plane k-1) and sE[en] are free
        load_ext_plane<TY>(sH[hn], H0, N, g, i0, j0, k + 1);
        __syncthreads();
        // E^n at plane k+1 (own cell, and the +x column / +y row)
        #pragma unroll 1
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1 && pex < 0) break;
            e_pos<TY>(g, sE[en], sH[hn], sH[hc], i0, j0, k + 1, pass ? pex : lane, pass ? pey : row,
                      pass == 0 && live && k + 1 < k1, E0, E1, eps, Eb0, store, qE, wave, grad);
        }
        __syncthreads();
        // H^{n-1/2} at plane k on the tile
        if (live) {
            const bool iI = x >= P && x < g.nx - P, jI = y >= P && y < g.ny - P, kI = k >= P && k < g.nz - P;
            const int idx = x + g.nx * (y + g.ny * k);
            if (iI && jI && kI) {
                const float exc = sE[ec][0][row][lane], eyc = sE[ec][1][row][lane], ezc = sE[ec][2][row][lane];
                H1[idx] = sH[hc][0][row + 1][lane + 1] +
                          dt * ((sE[ec][2][row + 1][lane] - ezc) - (sE[en][1][row][lane] - eyc));
                H1[N + idx] = sH[hc][1][row + 1][lane + 1] +
                              dt * ((sE[en][0][row][lane] - exc) - (sE[ec][2][row][lane + 1] - ezc));
                H1[2 * N + idx] = sH[hc][2][row + 1][lane + 1] +
                                  dt * ((sE[ec][1][row][lane + 1] - eyc) - (sE[ec][0][row + 1][lane] - exc));
            } else if (inject_h && P > 0) {
                // H^{n-1/2} on the low interface faces, for the next reverse step
                if (x == P - 1 && jI && kI) {
                    const int o = (k - P) * g.my + (y - P);
                    H1[N + idx] = shell_value(g, store, qH, 0, o);
                    H1[2 * N + idx] = shell_value(g, store, qH, 1, o);
                } else if (y == P - 1 && iI && kI) {
                    const int o = (k - P) * g.mx + (x - P);
                    H1[2 * N + idx] = shell_value(g, store, qH, 2, o);
                    H1[idx] = shell_value(g, store, qH, 3, o);
                } else if (k == P - 1 && iI && jI) {
                    const int o = (y - P) * g.mx + (x - P);
                    H1[idx] = shell_value(g, store, qH, 4, o);
                    H1[N + idx] = shell_value(g, store, qH, 5, o);
                }
            }
        }
        hc = hn;
        ec = en;
    }
}

// The recorded low-face H of the last step, injected into the final forward state.
__global__ __launch_bounds__(256) void k_inject_h(Grid g, float* __restrict__ H, const void* __restrict__ store,
                                                  Interp q) {
    const int P = g.P;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long ax = (long long)g.my * g.mz, ay = (long long)g.mx * g.mz, az = (long long)g.mx * g.my;
    const int N = (int)g.N;
    if (t < ax) {
        const int y = P + (int)(t % g.my), z = P + (int)(t / g.my), x = P - 1;
        const int idx = x + g.nx * (y + g.ny * z);
        H[N + idx] = shell_value(g, store, q, 0, t);
        H[2 * N + idx] = shell_value(g, store, q, 1, t);
    } else if (t < ax + ay) {
        const long long u = t - ax;
        const int x = P + (int)(u % g.mx), z = P + (int)(u / g.mx), y = P - 1;
        const int idx = x + g.nx * (y + g.ny * z);
        H[2 * N + idx] = shell_value(g, store, q, 2, u);
        H[idx] = shell_value(g, store, q, 3, u);
    } else if (t < ax + ay + az) {
        const long long u = t - ax - ay;
        const int x = P + (int)(u % g.mx), y = P + (int)(u / g.mx), z = P - 1;
        const int idx = x + g.nx * (y + g.ny * z);
        H[idx] = shell_value(g, store, q, 4, u);
        H[N + idx] = shell_value(g, store, q, 5, u);
    }
}

__global__ void k_scale_grad(double* g, long long n, const double* s) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[i] *= *s;
}

void launch_adj_step(const Grid& g, const Tiling& t, const float* Eb0, const float* Hb0, float* Eb1, float* Hb1,
                     const float* Es, const float* eps, const float* psi_in, float* psi_out, hipStream_t s) {
    if (t.ty == 8)
        launch_kernel(K_ADJ_STEP, k_adj_step<8>, dim3(t.count), dim3(TX, 8), s, g, t, Eb0, Hb0, Eb1, Hb1, Es, eps,
                      psi_in, psi_out);
    else
        launch_kernel(K_ADJ_STEP, k_adj_step<4>, dim3(t.count), dim3(TX, 4), s, g, t, Eb0, Hb0, Eb1, Hb1, Es, eps,
                      psi_in, psi_out);
}

void launch_prim_rev(const Grid& g, const Tiling& t, const int box_o[3], const int box_n[3], const float* E0,
                     const float* H0, float* E1, float* H1, const float* eps, const float* Eb0, const void* store,
                     Interp qE, Interp qH, int inject_h, float wave, double* grad, hipStream_t s) {
    Box b;
    for (int d = 0; d < 3; ++d) { b.o[d] = box_o[d]; b.n[d] = box_n[d]; }
    if (t.ty == 8)
        launch_kernel(K_PRIM_REV, k_prim_rev<8>, dim3(t.count), dim3(TX, 8), s, g, t, b, E0, H0, E1, H1, eps, Eb0,
                      store, qE, qH, inject_h, wave, grad);
    else
        launch_kernel(K_PRIM_REV, k_prim_rev<4>, dim3(t.count), dim3(TX, 4), s, g, t, b, E0, H0, E1, H1, eps, Eb0,
                      store, qE, qH, inject_h, wave, grad);
}

void launch_inject_h(const Grid& g, float* H, const void* store, Interp q, hipStream_t s) {
    if (g.P == 0) return;
    const long long n = (long long)g.my * g.mz + (long long)g.mx * g.mz + (long long)g.mx * g.my;
    launch_kernel(K_INJECT, k_inject_h, dim3((unsigned)((n + 255) / 256)), dim3(256), s, g, H, store, q);
}

void launch_scale_grad(double* grad, long long n, const double* scale, hipStream_t s) {
    if (n <= 0) return;
    launch_kernel(K_SCALE_GRAD, k_scale_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), s, grad, n, scale);
}

}  // namespace fdtd
