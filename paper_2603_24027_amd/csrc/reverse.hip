// Time-reversed gradient step (gfx950): primal reconstruction on the interior,
// interpolating reinjection of the recorded interface fields, the exact
// discrete adjoint of the CPML Yee step, and the FP64 dL/deps accumulator.
//
// Reverse step n (n = T-1 .. 0) is two sweeps:
//   rev_e  (undo the E half of forward step n)
//          primal : E^n = E^{n+1} - (dt/eps)(curl H^{n+1/2} - J^n) on the interior I
//                   (every interior node has PML depth 0, so no psi there);
//                   E^n on the high interface faces from the store (interpolated)
//          grad   : epsbar -= (dt/eps^2) sum_c Ebar_c (U_c - J_c) on the design box (FP64)
//          adjoint: v = (dt/eps) Ebar; per E-half term t = (c, d, s, f):
//                   P = psibar_t + s v_c,  gbar = s kinv_E v_c + a_E P,  psibar_t <- b_E P,
//                   Hbar_f += gbar(p) - gbar(p + e_d)
//   rev_h  (undo the H half of forward step n)
//          primal : H^{n-1/2} = H^{n+1/2} + dt curl E^n on I;
//                   H^{n-1/2} on the low interface faces from the store (for step n-1)
//          adjoint: w = -dt Hbar; per H-half term t = (c, d, s, f):
//                   P = psibar_t + s w_c,  gbar = s kinv_H w_c + a_H P,  psibar_t <- b_H P,
//                   Ebar_f += gbar(p - e_d) - gbar(p)
//          seed   : Ebar[D] += 2 E^n[D] for the loss term of E^n (n >= 1)
// Within one sweep no thread reads a value another thread writes: primal E is
// read only at the owner cell in rev_e, Ebar only read in rev_e and only
// written in rev_h (and the reverse for H, Hbar); the adjoint PML auxiliaries
// are read from one buffer and written to the other (ping-pong).
#include "common.h"

namespace fdtd {

struct TermCoef {
    const float* b;
    const float* a;
    const float* kinv;
};

// gbar of one term at a node: s kinv v + a (psibar + s v) inside the slab of its axis, s v outside.
__device__ inline float gbar_term(float sv, int sc, const TermCoef& c, const float* psi, long long o) {
    if (sc < 0) return sv;
    return c.kinv[sc] * sv + c.a[sc] * (psi[o] + sv);
}

__device__ inline long long slab_index(const Grid& g, int axis, int i, int j, int k, int s) {
    if (axis == 0) return s + 2LL * g.P * (j + (long long)g.ny * k);
    if (axis == 1) return i + (long long)g.nx * (s + 2LL * g.P * k);
    return i + (long long)g.nx * (j + (long long)g.ny * s);
}

__global__ __launch_bounds__(BX * BY) void k_rev_init(Grid g, float* __restrict__ F, float* __restrict__ A,
                                                      const void* __restrict__ store, Interp q) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long N = g.N;
    const long long idx = i + (long long)g.nx * (j + (long long)g.ny * k);
    const bool det = in_box(i, j, k, g.det_lo, g.det_hi);
    for (int c = 0; c < 3; ++c) A[c * N + idx] = det ? 2.0f * F[c * N + idx] : 0.0f;   // seed from E^T
    for (int c = 3; c < 6; ++c) A[c * N + idx] = 0.0f;
    const int P = g.P;
    if (P == 0) return;
    const bool jI = j >= P && j < g.ny - P, kI = k >= P && k < g.nz - P, iI = i >= P && i < g.nx - P;
    float* Hx = F + 3 * N;
    float* Hy = F + 4 * N;
    float* Hz = F + 5 * N;
    if (i == P - 1 && jI && kI) {
        long long off = (long long)(k - P) * g.my + (j - P);
        Hy[idx] = shell_value(g, store, q, 0, off);
        Hz[idx] = shell_value(g, store, q, 1, off);
    }
    if (j == P - 1 && iI && kI) {
        long long off = (long long)(k - P) * g.mx + (i - P);
        Hz[idx] = shell_value(g, store, q, 2, off);
        Hx[idx] = shell_value(g, store, q, 3, off);
    }
    if (k == P - 1 && iI && jI) {
        long long off = (long long)(j - P) * g.mx + (i - P);
        Hx[idx] = shell_value(g, store, q, 4, off);
        Hy[idx] = shell_value(g, store, q, 5, off);
    }
}

__global__ __launch_bounds__(BX * BY) void k_rev_e(Grid g, float* __restrict__ F, const float* __restrict__ eps,
                                                   float* __restrict__ A, const float* __restrict__ psi_in,
                                                   float* __restrict__ psi_out, const void* __restrict__ store,
                                                   Interp q, float wave, double* __restrict__ grad) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long N = g.N;
    const long long sy = g.nx, sz = (long long)g.nx * g.ny;
    const long long idx = i + sy * j + sz * k;
    const int P = g.P;
    const float dt = g.dt;
    const bool iI = i >= P && i < g.nx - P, jI = j >= P && j < g.ny - P, kI = k >= P && k < g.nz - P;

    const float* Ebx = A;
    const float* Eby = A + N;
    const float* Ebz = A + 2 * N;
    const float ebx = Ebx[idx], eby = Eby[idx], ebz = Ebz[idx];
    const float ce = dt / eps[idx];

    // ---- primal: E^{n+1} -> E^n on the interior; gradient on the design box ----
    if (iI && jI && kI) {
        const float* Hx = F + 3 * N;
        const float* Hy = F + 4 * N;
        const float* Hz = F + 5 * N;
        const float hx = Hx[idx], hy = Hy[idx], hz = Hz[idx];
        const int pr = g.periodic;
        float ux = (hz - nb_minus(Hz, idx, j, g.ny, sy, pr)) - (hy - nb_minus(Hy, idx, k, g.nz, sz, pr));
        float uy = (hx - nb_minus(Hx, idx, k, g.nz, sz, pr)) - (hz - nb_minus(Hz, idx, i, g.nx, 1, pr));
        float uz = (hy - nb_minus(Hy, idx, i, g.nx, 1, pr)) - (hx - nb_minus(Hx, idx, j, g.ny, sy, pr));
        if (in_box(i, j, k, g.src_lo, g.src_hi)) {
            const int sxn = g.src_hi[0] - g.src_lo[0], syn = g.src_hi[1] - g.src_lo[1];
            const float jv = wave * g.src_profile[(i - g.src_lo[0]) + (long long)sxn *
                                                  ((j - g.src_lo[1]) + (long long)syn * (k - g.src_lo[2]))];
            if (g.src_comp == 0) ux -= jv; else if (g.src_comp == 1) uy -= jv; else uz -= jv;
        }
        float* Ex = F;
        float* Ey = F + N;
        float* Ez = F + 2 * N;
        Ex[idx] -= ce * ux;
        Ey[idx] -= ce * uy;
        Ez[idx] -= ce * uz;
        if (in_box(i, j, k, g.des_lo, g.des_hi)) {
            const int dx = g.des_hi[0] - g.des_lo[0], dy = g.des_hi[1] - g.des_lo[1];
            const long long di = (i - g.des_lo[0]) + (long long)dx * ((j - g.des_lo[1]) + (long long)dy * (k - g.des_lo[2]));
            const double e = (double)eps[idx];
            const double s = (double)ebx * ux + (double)eby * uy + (double)ebz * uz;
            grad[di] -= (double)dt / (e * e) * s;
        }
    } else if (P > 0) {
        // E^n on the high interface faces
        float* Ex = F;
        float* Ey = F + N;
        float* Ez = F + 2 * N;
        if (i == g.nx - P && jI && kI) {
            long long off = (long long)(k - P) * g.my + (j - P);
            Ey[idx] = shell_value(g, store, q, 6, off);
            Ez[idx] = shell_value(g, store, q, 7, off);
        }
        if (j == g.ny - P && iI && kI) {
            long long off = (long long)(k - P) * g.mx + (i - P);
            Ez[idx] = shell_value(g, store, q, 8, off);
            Ex[idx] = shell_value(g, store, q, 9, off);
        }
        if (k == g.nz - P && iI && jI) {
            long long off = (long long)(j - P) * g.mx + (i - P);
            Ex[idx] = shell_value(g, store, q, 10, off);
            Ey[idx] = shell_value(g, store, q, 11, off);
        }
    }

    // ---- adjoint of the E half ----
    const TermCoef cE = {g.coef, g.coef + 2 * P, g.coef + 4 * P};
    const float vx = ce * ebx, vy = ce * eby, vz = ce * ebz;
    // own node: gbar for the six terms, and psibar updates
    const int sxo = P > 0 ? slab_coord(i, g.nx, P) : -1;
    const int syo = P > 0 ? slab_coord(j, g.ny, P) : -1;
    const int szo = P > 0 ? slab_coord(k, g.nz, P) : -1;
    // term -> (v, sign, axis):  0 (vx,+,y) 1 (vx,-,z) 2 (vy,+,z) 3 (vy,-,x) 4 (vz,+,x) 5 (vz,-,y)
    float g0, g1, g2, g3, g4, g5;
    {
        const float s0 = vx, s1 = -vx, s2 = vy, s3 = -vy, s4 = vz, s5 = -vz;
        g0 = s0; g5 = s5; g1 = s1; g2 = s2; g3 = s3; g4 = s4;
        if (sxo >= 0) {
            const long long o = g.psi_off[0] + 2 * g.slab[0] + slab_index(g, 0, i, j, k, sxo);
            const float Pa = psi_in[o] + s3, Pb = psi_in[o + g.slab[0]] + s4;
            g3 = cE.kinv[sxo] * s3 + cE.a[sxo] * Pa;
            g4 = cE.kinv[sxo] * s4 + cE.a[sxo] * Pb;
            psi_out[o] = cE.b[sxo] * Pa;
            psi_out[o + g.slab[0]] = cE.b[sxo] * Pb;
        }
        if (syo >= 0) {
            const long long o = g.psi_off[1] + 2 * g.slab[1] + slab_index(g, 1, i, j, k, syo);
            const float Pa = psi_in[o] + s0, Pb = psi_in[o + g.slab[1]] + s5;
            g0 = cE.kinv[syo] * s0 + cE.a[syo] * Pa;
            g5 = cE.kinv[syo] * s5 + cE.a[syo] * Pb;
            psi_out[o] = cE.b[syo] * Pa;
            psi_out[o + g.slab[1]] = cE.b[syo] * Pb;
        }
        if (szo >= 0) {
            const long long o = g.psi_off[2] + 2 * g.slab[2] + slab_index(g, 2, i, j, k, szo);
            const float Pa = psi_in[o] + s1, Pb = psi_in[o + g.slab[2]] + s2;
            g1 = cE.kinv[szo] * s1 + cE.a[szo] * Pa;
            g2 = cE.kinv[szo] * s2 + cE.a[szo] * Pb;
            psi_out[o] = cE.b[szo] * Pa;
            psi_out[o + g.slab[2]] = cE.b[szo] * Pb;
        }
    }
    // neighbours at +x (terms 3, 4), +y (terms 0, 5), +z (terms 1, 2)
    float n3 = 0.f, n4 = 0.f, n0 = 0.f, n5 = 0.f, n1 = 0.f, n2 = 0.f;
    {
        const bool has = (i + 1 < g.nx) || g.periodic;
        if (has) {
            const int ii = (i + 1 < g.nx) ? i + 1 : 0;
            const long long id2 = idx + (ii - i);
            const float c2 = dt / eps[id2];
            const float s3 = -c2 * Eby[id2], s4 = c2 * Ebz[id2];
            const int sc = P > 0 ? slab_coord(ii, g.nx, P) : -1;
            const long long o = g.psi_off[0] + 2 * g.slab[0] + (sc >= 0 ? slab_index(g, 0, ii, j, k, sc) : 0);
            n3 = gbar_term(s3, sc, cE, psi_in, o);
            n4 = gbar_term(s4, sc, cE, psi_in, o + g.slab[0]);
        }
    }
    {
        const bool has = (j + 1 < g.ny) || g.periodic;
        if (has) {
            const int jj = (j + 1 < g.ny) ? j + 1 : 0;
            const long long id2 = idx + (long long)(jj - j) * sy;
            const float c2 = dt / eps[id2];
            const float s0 = c2 * Ebx[id2], s5 = -c2 * Ebz[id2];
            const int sc = P > 0 ? slab_coord(jj, g.ny, P) : -1;
            const long long o = g.psi_off[1] + 2 * g.slab[1] + (sc >= 0 ? slab_index(g, 1, i, jj, k, sc) : 0);
            n0 = gbar_term(s0, sc, cE, psi_in, o);
            n5 = gbar_term(s5, sc, cE, psi_in, o + g.slab[1]);
        }
    }
    {
        const bool has = (k + 1 < g.nz) || g.periodic;
        if (has) {
            const int kk = (k + 1 < g.nz) ? k + 1 : 0;
            const long long id2 = idx + (long long)(kk - k) * sz;
            const float c2 = dt / eps[id2];
            const float s1 = -c2 * Ebx[id2], s2 = c2 * Eby[id2];
            const int sc = P > 0 ? slab_coord(kk, g.nz, P) : -1;
            const long long o = g.psi_off[2] + 2 * g.slab[2] + (sc >= 0 ? slab_index(g, 2, i, j, kk, sc) : 0);
            n1 = gbar_term(s1, sc, cE, psi_in, o);
            n2 = gbar_term(s2, sc, cE, psi_in, o + g.slab[2]);
        }
    }
    float* Hbx = A + 3 * N;
    float* Hby = A + 4 * N;
    float* Hbz = A + 5 * N;
    // Hx <- terms 2 (z) and 5 (y); Hy <- 1 (z) and 4 (x); Hz <- 0 (y) and 3 (x)
    Hbx[idx] += (g2 - n2) + (g5 - n5);
    Hby[idx] += (g1 - n1) + (g4 - n4);
    Hbz[idx] += (g0 - n0) + (g3 - n3);
}

__global__ __launch_bounds__(BX * BY) void k_rev_h(Grid g, float* __restrict__ F, float* __restrict__ A,
                                                   const float* __restrict__ psi_in, float* __restrict__ psi_out,
                                                   const void* __restrict__ store, Interp q, int inject,
                                                   int seed) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long N = g.N;
    const long long sy = g.nx, sz = (long long)g.nx * g.ny;
    const long long idx = i + sy * j + sz * k;
    const int P = g.P;
    const float dt = g.dt;
    const bool iI = i >= P && i < g.nx - P, jI = j >= P && j < g.ny - P, kI = k >= P && k < g.nz - P;

    // ---- primal: H^{n+1/2} -> H^{n-1/2} on I; low interface faces for the next reverse step ----
    const float* Ex = F;
    const float* Ey = F + N;
    const float* Ez = F + 2 * N;
    float* Hx = F + 3 * N;
    float* Hy = F + 4 * N;
    float* Hz = F + 5 * N;
    if (iI && jI && kI) {
        const float ex = Ex[idx], ey = Ey[idx], ez = Ez[idx];
        const int pr = g.periodic;
        Hx[idx] += dt * ((nb_plus(Ez, idx, j, g.ny, sy, pr) - ez) - (nb_plus(Ey, idx, k, g.nz, sz, pr) - ey));
        Hy[idx] += dt * ((nb_plus(Ex, idx, k, g.nz, sz, pr) - ex) - (nb_plus(Ez, idx, i, g.nx, 1, pr) - ez));
        Hz[idx] += dt * ((nb_plus(Ey, idx, i, g.nx, 1, pr) - ey) - (nb_plus(Ex, idx, j, g.ny, sy, pr) - ex));
    } else if (inject && P > 0) {
        if (i == P - 1 && jI && kI) {
            long long off = (long long)(k - P) * g.my + (j - P);
            Hy[idx] = shell_value(g, store, q, 0, off);
            Hz[idx] = shell_value(g, store, q, 1, off);
        }
        if (j == P - 1 && iI && kI) {
            long long off = (long long)(k - P) * g.mx + (i - P);
            Hz[idx] = shell_value(g, store, q, 2, off);
            Hx[idx] = shell_value(g, store, q, 3, off);
        }
        if (k == P - 1 && iI && jI) {
            long long off = (long long)(j - P) * g.mx + (i - P);
            Hx[idx] = shell_value(g, store, q, 4, off);
            Hy[idx] = shell_value(g, store, q, 5, off);
        }
    }

    // ---- adjoint of the H half ----
    const TermCoef cH = {g.coef + 6 * P, g.coef + 8 * P, g.coef + 10 * P};
    const float* Hbx = A + 3 * N;
    const float* Hby = A + 4 * N;
    const float* Hbz = A + 5 * N;
    const float wx = -dt * Hbx[idx], wy = -dt * Hby[idx], wz = -dt * Hbz[idx];
    const int sxo = P > 0 ? slab_coord(i, g.nx, P) : -1;
    const int syo = P > 0 ? slab_coord(j, g.ny, P) : -1;
    const int szo = P > 0 ? slab_coord(k, g.nz, P) : -1;
    // term -> (w, sign, axis): 0 (wx,+,y) 1 (wx,-,z) 2 (wy,+,z) 3 (wy,-,x) 4 (wz,+,x) 5 (wz,-,y)
    float g0 = wx, g1 = -wx, g2 = wy, g3 = -wy, g4 = wz, g5 = -wz;
    if (sxo >= 0) {
        const long long o = g.psi_off[0] + slab_index(g, 0, i, j, k, sxo);
        const float Pa = psi_in[o] + g3, Pb = psi_in[o + g.slab[0]] + g4;
        const float s3 = g3, s4 = g4;
        g3 = cH.kinv[sxo] * s3 + cH.a[sxo] * Pa;
        g4 = cH.kinv[sxo] * s4 + cH.a[sxo] * Pb;
        psi_out[o] = cH.b[sxo] * Pa;
        psi_out[o + g.slab[0]] = cH.b[sxo] * Pb;
    }
    if (syo >= 0) {
        const long long o = g.psi_off[1] + slab_index(g, 1, i, j, k, syo);
        const float Pa = psi_in[o] + g0, Pb = psi_in[o + g.slab[1]] + g5;
        const float s0 = g0, s5 = g5;
        g0 = cH.kinv[syo] * s0 + cH.a[syo] * Pa;
        g5 = cH.kinv[syo] * s5 + cH.a[syo] * Pb;
        psi_out[o] = cH.b[syo] * Pa;
        psi_out[o + g.slab[1]] = cH.b[syo] * Pb;
    }
    if (szo >= 0) {
        const long long o = g.psi_off[2] + slab_index(g, 2, i, j, k, szo);
        const float Pa = psi_in[o] + g1, Pb = psi_in[o + g.slab[2]] + g2;
        const float s1 = g1, s2 = g2;
        g1 = cH.kinv[szo] * s1 + cH.a[szo] * Pa;
        g2 = cH.kinv[szo] * s2 + cH.a[szo] * Pb;
        psi_out[o] = cH.b[szo] * Pa;
        psi_out[o + g.slab[2]] = cH.b[szo] * Pb;
    }
    // neighbours at -x (terms 3, 4), -y (terms 0, 5), -z (terms 1, 2)
    float n3 = 0.f, n4 = 0.f, n0 = 0.f, n5 = 0.f, n1 = 0.f, n2 = 0.f;
    if (i > 0 || g.periodic) {
        const int ii = i > 0 ? i - 1 : g.nx - 1;
        const long long id2 = idx + (ii - i);
        const float s3 = dt * Hby[id2], s4 = -dt * Hbz[id2];   // -w_y, +w_z
        const int sc = P > 0 ? slab_coord(ii, g.nx, P) : -1;
        const long long o = g.psi_off[0] + (sc >= 0 ? slab_index(g, 0, ii, j, k, sc) : 0);
        n3 = gbar_term(s3, sc, cH, psi_in, o);
        n4 = gbar_term(s4, sc, cH, psi_in, o + g.slab[0]);
    }
    if (j > 0 || g.periodic) {
        const int jj = j > 0 ? j - 1 : g.ny - 1;
        const long long id2 = idx + (long long)(jj - j) * sy;
        const float s0 = -dt * Hbx[id2], s5 = dt * Hbz[id2];   // +w_x, -w_z
        const int sc = P > 0 ? slab_coord(jj, g.ny, P) : -1;
        const long long o = g.psi_off[1] + (sc >= 0 ? slab_index(g, 1, i, jj, k, sc) : 0);
        n0 = gbar_term(s0, sc, cH, psi_in, o);
        n5 = gbar_term(s5, sc, cH, psi_in, o + g.slab[1]);
    }
    if (k > 0 || g.periodic) {
        const int kk = k > 0 ? k - 1 : g.nz - 1;
        const long long id2 = idx + (long long)(kk - k) * sz;
        const float s1 = dt * Hbx[id2], s2 = -dt * Hby[id2];   // -w_x, +w_y
        const int sc = P > 0 ? slab_coord(kk, g.nz, P) : -1;
        const long long o = g.psi_off[2] + (sc >= 0 ? slab_index(g, 2, i, j, kk, sc) : 0);
        n1 = gbar_term(s1, sc, cH, psi_in, o);
        n2 = gbar_term(s2, sc, cH, psi_in, o + g.slab[2]);
    }
    float* Ebx = A;
    float* Eby = A + N;
    float* Ebz = A + 2 * N;
    // Ex <- terms 2 (z) and 5 (y); Ey <- 1 (z) and 4 (x); Ez <- 0 (y) and 3 (x)
    float ebx = Ebx[idx] + (n2 - g2) + (n5 - g5);
    float eby = Eby[idx] + (n1 - g1) + (n4 - g4);
    float ebz = Ebz[idx] + (n0 - g0) + (n3 - g3);
    if (seed && in_box(i, j, k, g.det_lo, g.det_hi)) {
        ebx += 2.0f * Ex[idx];
        eby += 2.0f * Ey[idx];
        ebz += 2.0f * Ez[idx];
    }
    Ebx[idx] = ebx;
    Eby[idx] = eby;
    Ebz[idx] = ebz;
}

__global__ void k_scale_grad(double* g, long long n, const double* s) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[i] *= *s;
}

static dim3 grid_dims(const Grid& g) {
    return dim3((unsigned)((g.nx + BX - 1) / BX), (unsigned)((g.ny + BY - 1) / BY), (unsigned)g.nz);
}

void launch_rev_init(const Grid& g, float* fields, float* adj, const void* store, Interp q, hipStream_t s) {
    launch_kernel(K_REV_INIT, k_rev_init, grid_dims(g), dim3(BX, BY), s, g, fields, adj, store, q);
}

void launch_rev_e(const Grid& g, float* fields, const float* eps, float* adj, const float* psi_in,
                  float* psi_out, const void* store, Interp q, float wave, double* grad, hipStream_t s) {
    launch_kernel(K_REV_E, k_rev_e, grid_dims(g), dim3(BX, BY), s, g, fields, eps, adj, psi_in, psi_out, store, q,
                       wave, grad);
}

void launch_rev_h(const Grid& g, float* fields, float* adj, const float* psi_in, float* psi_out,
                  const void* store, Interp q, int inject, int seed, hipStream_t s) {
    launch_kernel(K_REV_H, k_rev_h, grid_dims(g), dim3(BX, BY), s, g, fields, adj, psi_in, psi_out, store, q,
                       inject, seed);
}

void launch_scale_grad(double* grad, long long n, const double* scale, hipStream_t s) {
    if (n <= 0) return;
    launch_kernel(K_SCALE_GRAD, k_scale_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), s, grad, n, scale);
}

}  // namespace fdtd
