// Two reverse steps of the primal interior per sweep (temporal blocking of the reversal, gfx950).
//
// One sweep takes (E^{n+1}, H^{n+1/2}) in F0 to (E^{n-1}, H^{n-3/2}) in F1 on the lossless
// interior I (every interior node has PML depth 0), undoing forward steps n and n-1 with
// the arithmetic of the single-step reversal (reverse.hip), twice:
//   E^m       = E^{m+1} - (dt/eps)(curl H^{m+1/2} - J^m)    (backward differences)
//   H^{m-1/2} = H^{m+1/2} + dt curl E^m                     (forward differences)
// (Section 1: backwards from the final step; Section 2: the recorded interface fields act
// as sources).  The interface shell of the two steps comes from three places:
//   * F0 holds the input state's H^{n+1/2} on the low faces and the second step's
//     E^{n-1} on the high faces (positions whose E no interior update writes);
//   * F1 holds the second step's H^{n-3/2} on the low faces (the next sweep reads it);
//   * the first step's E^n (high faces) and H^{n-1/2} (low faces), which no field buffer
//     can hold beside those, sit in `mid`, laid out as one kept step of the store; each
//     tile that meets a face copies its part into LDS before it marches.
// Step n's loss seed and gradient term are taken as in the single-step reversal (the
// adjoint state of step n is in Eb0).  Step n-1's need the adjoint state after step n's
// transpose, which the adjoint sweep produces later: the sweep keeps E^n and H^{n-1/2} of
// the detector cells and curl H^{n-1/2} - J^{n-1} and eps of the design cells in `stash`,
// and k_rev_pending applies them after that transpose.
//
// Geometry as in the two-step forward (forward2.hip), mirrored.  A block owns 60 x HY
// interior columns and CZ planes; its 64 x (HY + 4) threads cover two more cells on each
// side in x and y.  Valid regions around the owned tile: E^n on [-1, +2], H^{n-1/2} on
// [-1, +1], E^{n-1} on [0, +1], H^{n-3/2} the tile.  Iteration j evaluates E^n(j) and
// H^{n-1/2}(j-1), then E^{n-1}(j-1) and H^{n-3/2}(j-2), with one LDS plane per field:
//   E^n(j), H^{n-1/2}(j-1) -> sHA; E^{n-1}(j-2) -> sEB | A | E^{n-1}(j-1), H^{n-3/2}(j-2);
//   H^{n+1/2}(j+1) -> sHin, E^n(j) -> sEA | B.
#include "march.h"

namespace fdtd {

template <int HY>
using RPlane = float[3][HY + 6][TX + 2];   // one LDS plane, padded by one cell on every side

// The intermediate shell of a tile in LDS: [side 0 E / 1 H][tangential component] per face.
// x faces: (row, plane); y faces: (lane, plane); z faces: (row, lane).
template <int HY, int CZ>
struct ShellTile {
    float x[2][2][HY + 4][CZ + 3];
    float y[2][2][TX][CZ + 3];
    float z[2][2][HY + 4][TX];
};

struct Rev2Bufs {
    rsrc_t F0, F1, eps, src;
};

// Inputs of iteration j, loaded one iteration ahead: H^{n+1/2}(j+1) (published to LDS at
// the end of iteration j), E(j) from F0 (E^{n+1} on I, E^{n-1} on the high faces), eps(j),
// the source profile at j.
struct RIn {
    float h[3], e[3], ep, sp;
};

struct Rev2Ctx {
    int lane, row, x, y, plane, k0, k1;
    bool live, own, inxy;
    bool xhe, xlh, yhe, ylh;   // on the x / y high (E) or low (H) face, within the face's extent
    uint32_t f, o, src;         // lane offsets: column loads, owned stores, source box column
    uint32_t nb;
};

__device__ inline bool zin(const Grid& g, int z) { return z >= g.P && z < g.nz - g.P; }

template <int HY, int CZ>
__device__ __forceinline__ void load_rin(const Grid& g, const Rev2Bufs& b, const Rev2Ctx& c, int j, RIn& d) {
    const int zj = bound(j, g.nz, g.periodic), z1 = bound(j + 1, g.nz, g.periodic);
    const uint32_t s1 = uni(z1 < 0 ? 0u : (uint32_t)(z1 * c.plane) << 2);
    bld3v(b.F0, z1 < 0 ? OOB : c.f, s1 + 3 * c.nb, c.nb, d.h);
    const uint32_t sj = uni(zj < 0 ? 0u : (uint32_t)(zj * c.plane) << 2);
    const uint32_t vj = zj < 0 ? OOB : c.f;
    bld3v(b.F0, vj, sj, c.nb, d.e);
    const float ep = bldv(b.eps, vj, sj);
    d.ep = (c.live && zj >= 0) ? ep : 1.0f;
    uint32_t ss = 0;
    const bool sin = zj >= 0 && zj >= g.src_lo[2] && zj < g.src_hi[2];
    if (sin) ss = (uint32_t)((zj - g.src_lo[2]) * (g.src_hi[0] - g.src_lo[0]) * (g.src_hi[1] - g.src_lo[1])) << 2;
    d.sp = bldv(b.src, sin ? c.src : OOB, uni(ss));
}

// index of a cell in a box, or -1 outside
__device__ inline long long box_index(int x, int y, int z, const int lo[3], const int hi[3]) {
    if (!in_box(x, y, z, lo, hi)) return -1;
    return (x - lo[0]) + (long long)(hi[0] - lo[0]) * ((y - lo[1]) + (long long)(hi[1] - lo[1]) * (z - lo[2]));
}

// Whether a cell of this thread's column on plane z lies on a face of side s (0: the high
// faces, where E is recorded; 1: the low faces, where H is), within the face's extent.
__device__ __forceinline__ bool on_face(const Grid& g, const Rev2Ctx& c, int s, int z) {
    if (g.P == 0) return false;
    const bool zi = zin(g, z);
    if (zi && (s == 0 ? (c.xhe || c.yhe) : (c.xlh || c.ylh))) return true;
    return c.inxy && z == (s == 0 ? g.nz - g.P : g.P - 1);
}

// The intermediate shell value of side `s` (0: E on the high faces, 1: H on the low faces)
// at a cell of this thread's column on plane z, as three components (the normal one 0);
// false when the cell is on no face of that side.
template <int HY, int CZ>
__device__ __forceinline__ bool shell_at(const Grid& g, const ShellTile<HY, CZ>& st, const Rev2Ctx& c, int s, int z,
                                         int jj, float v[3]) {
    const bool zi = zin(g, z);
    if (zi && (s == 0 ? c.xhe : c.xlh)) {          // x face: (y, z) components
        v[0] = 0.0f; v[1] = st.x[s][0][c.row][jj]; v[2] = st.x[s][1][c.row][jj];
        return true;
    }
    if (zi && (s == 0 ? c.yhe : c.ylh)) {          // y face: (z, x) components
        v[0] = st.y[s][1][c.lane][jj]; v[1] = 0.0f; v[2] = st.y[s][0][c.lane][jj];
        return true;
    }
    if (c.inxy && g.P > 0 && z == (s == 0 ? g.nz - g.P : g.P - 1)) {   // z face: (x, y) components
        v[0] = st.z[s][0][c.row][c.lane]; v[1] = st.z[s][1][c.row][c.lane]; v[2] = 0.0f;
        return true;
    }
    return false;
}

// Copy the tile's part of the intermediate shell from mid into LDS (all threads; a
// barrier follows).  Rows/lanes/planes off a face's extent read 0.
template <int HY, int CZ>
__device__ inline void fill_shell_tile(const Grid& g, ShellTile<HY, CZ>& st, const float* __restrict__ mid, int a,
                                       int j0, int k0, int tid, int nthreads) {
    const int P = g.P;
    constexpr int NXF = 2 * 2 * (HY + 4) * (CZ + 3), NYF = 2 * 2 * TX * (CZ + 3), NZF = 2 * 2 * (HY + 4) * TX;
    for (int e = tid; e < NXF + NYF + NZF; e += nthreads) {
        float v = 0.0f;
        if (e < NXF) {
            const int s = e / (2 * (HY + 4) * (CZ + 3)), q = (e / ((HY + 4) * (CZ + 3))) % 2;
            const int r = (e / (CZ + 3)) % (HY + 4), jj = e % (CZ + 3);
            const int y = j0 - 2 + r, z = k0 - 1 + jj;
            if (y >= P && y < g.ny - P && z >= P && z < g.nz - P)
                v = mid[block_offset(g, (s == 0 ? 6 : 0) + q) + (y - P) + (long long)g.my * (z - P)];
            st.x[s][q][r][jj] = v;
        } else if (e < NXF + NYF) {
            const int r0 = e - NXF;
            const int s = r0 / (2 * TX * (CZ + 3)), q = (r0 / (TX * (CZ + 3))) % 2;
            const int l = (r0 / (CZ + 3)) % TX, jj = r0 % (CZ + 3);
            const int x = a - 2 + l, z = k0 - 1 + jj;
            if (x >= P && x < g.nx - P && z >= P && z < g.nz - P)
                v = mid[block_offset(g, (s == 0 ? 8 : 2) + q) + (x - P) + (long long)g.mx * (z - P)];
            st.y[s][q][l][jj] = v;
        } else {
            const int r0 = e - NXF - NYF;
            const int s = r0 / (2 * (HY + 4) * TX), q = (r0 / ((HY + 4) * TX)) % 2;
            const int r = (r0 / TX) % (HY + 4), l = r0 % TX;
            const int x = a - 2 + l, y = j0 - 2 + r;
            if (x >= P && x < g.nx - P && y >= P && y < g.ny - P)
                v = mid[block_offset(g, (s == 0 ? 10 : 4) + q) + (x - P) + (long long)g.mx * (y - P)];
            st.z[s][q][r][l] = v;
        }
    }
}

// State carried from iteration j-1 to j (the thread's own column).
struct RCarry {
    float h0p[3];   // H^{n+1/2}(j-1)
    float e0p[3];   // E from F0 at j-1 (E^{n-1} on the high faces)
    float ha[3];    // H^{n-1/2}(j-2)
    float eb[3];    // E^{n-1}(j-2), published to LDS at the start of iteration j
    float ep, sp;   // eps(j-1), source profile at j-1
};

template <int HY, int CZ, bool FACES>
__device__ __forceinline__ void iter_rev2(const Grid& g, const Rev2Bufs& b, const Rev2Ctx& c, RPlane<HY>& sHin,
                                          RPlane<HY>& sEA, RPlane<HY>& sHA, RPlane<HY>& sEB,
                                          const ShellTile<HY, CZ>& st, int j, const RIn& in, RCarry& cr, float w0,
                                          float w1, float* __restrict__ Eb0, double* __restrict__ grad,
                                          float* __restrict__ stash) {
    const int lane = c.lane, row = c.row, lx = lane + 1, ly = row + 1;
    const int jj = j - (c.k0 - 1), jjp = jj > 0 ? jj - 1 : 0;
    const int zj = bound(j, g.nz, g.periodic), zp = bound(j - 1, g.nz, g.periodic), zq = bound(j - 2, g.nz, g.periodic);
    const bool zjI = zj >= 0 && zin(g, zj), zpI = zp >= 0 && zin(g, zp), zqI = zq >= 0 && zin(g, zq);
    const bool inj = c.live && c.inxy && zjI, inp = c.live && c.inxy && zpI, inq = c.live && c.inxy && zqI;
    const bool own1 = c.own && j >= c.k0 && j < c.k1;            // plane j is one of the block's own
    const bool own2 = c.own && j - 1 >= c.k0 && j - 1 < c.k1;    // plane j-1
    const bool own3 = c.own && j - 2 >= c.k0 && j - 2 < c.k1;    // plane j-2
    const float dt = g.dt;
    const uint32_t nb = c.nb;
    // ---- E^n(j) ----
    float ea[3];
    const float hx = sHin[0][ly][lx], hy = sHin[1][ly][lx], hz = sHin[2][ly][lx];   // H^{n+1/2}(j), own
    {
        float u[3];
        u[0] = (hz - sHin[2][ly - 1][lx]) - (hy - cr.h0p[1]);
        u[1] = (hx - cr.h0p[0]) - (hz - sHin[2][ly][lx - 1]);
        u[2] = (hy - sHin[1][ly][lx - 1]) - (hx - sHin[0][ly - 1][lx]);
        const float jv = w0 * in.sp;
        u[0] -= g.src_comp == 0 ? jv : 0.0f;
        u[1] -= g.src_comp == 1 ? jv : 0.0f;
        u[2] -= g.src_comp == 2 ? jv : 0.0f;
        const float cc = dt_over_eps(dt, in.ep);
        ea[0] = inj ? in.e[0] - cc * u[0] : 0.0f;
        ea[1] = inj ? in.e[1] - cc * u[1] : 0.0f;
        ea[2] = inj ? in.e[2] - cc * u[2] : 0.0f;
        if constexpr (FACES) {
            float v[3];
            if (!inj && c.live && zj >= 0 && shell_at<HY, CZ>(g, st, c, 0, zj, jj, v)) { ea[0] = v[0]; ea[1] = v[1]; ea[2] = v[2]; }
        }
        if (own1 && inj) {
            const float h[3] = {hx, hy, hz};
            grad_and_seed(g, Eb0, grad, c.x, c.y, zj, (int)((long long)(c.x + g.nx * c.y) + (long long)zj * c.plane),
                          in.e, h, in.ep, u);
        }
    }
    // ---- H^{n-1/2}(j-1) ----
    float ha[3];
    {
        const float ex = sEA[0][ly][lx], ey = sEA[1][ly][lx], ez = sEA[2][ly][lx];   // E^n(j-1), own
        ha[0] = inp ? cr.h0p[0] + dt * ((sEA[2][ly + 1][lx] - ez) - (ea[1] - ey)) : 0.0f;
        ha[1] = inp ? cr.h0p[1] + dt * ((ea[0] - ex) - (sEA[2][ly][lx + 1] - ez)) : 0.0f;
        ha[2] = inp ? cr.h0p[2] + dt * ((sEA[1][ly][lx + 1] - ey) - (sEA[0][ly + 1][lx] - ex)) : 0.0f;
        if constexpr (FACES) {
            float v[3];
            if (!inp && c.live && zp >= 0 && shell_at<HY, CZ>(g, st, c, 1, zp, jjp, v)) { ha[0] = v[0]; ha[1] = v[1]; ha[2] = v[2]; }
        }
        if (own2 && inp) {   // step n-1's seed needs E^n and H^{n-1/2} on the detector
            const long long di = box_index(c.x, c.y, zp, g.det_lo, g.det_hi);
            if (di >= 0) {
                float* q = stash + 6 * di;
                q[0] = ex; q[1] = ey; q[2] = ez; q[3] = ha[0]; q[4] = ha[1]; q[5] = ha[2];
            }
        }
    }
    sHA[0][ly][lx] = ha[0];
    sHA[1][ly][lx] = ha[1];
    sHA[2][ly][lx] = ha[2];
    sEB[0][ly][lx] = cr.eb[0];
    sEB[1][ly][lx] = cr.eb[1];
    sEB[2][ly][lx] = cr.eb[2];
    __syncthreads();   // A
    // ---- E^{n-1}(j-1) ----
    float eb[3];
    {
        float u[3];
        u[0] = (ha[2] - sHA[2][ly - 1][lx]) - (ha[1] - cr.ha[1]);
        u[1] = (ha[0] - cr.ha[0]) - (ha[2] - sHA[2][ly][lx - 1]);
        u[2] = (ha[1] - sHA[1][ly][lx - 1]) - (ha[0] - sHA[0][ly - 1][lx]);
        const float jv = w1 * cr.sp;
        u[0] -= g.src_comp == 0 ? jv : 0.0f;
        u[1] -= g.src_comp == 1 ? jv : 0.0f;
        u[2] -= g.src_comp == 2 ? jv : 0.0f;
        const float cc = dt_over_eps(dt, cr.ep);
        const float e0 = sEA[0][ly][lx], e1 = sEA[1][ly][lx], e2 = sEA[2][ly][lx];   // E^n(j-1), own
        eb[0] = inp ? e0 - cc * u[0] : 0.0f;
        eb[1] = inp ? e1 - cc * u[1] : 0.0f;
        eb[2] = inp ? e2 - cc * u[2] : 0.0f;
        if constexpr (FACES) {
            // high faces: the recorded E^{n-1}, read from F0 with the rest of plane j-1
            if (!inp && c.live && zp >= 0 && on_face(g, c, 0, zp)) {
                eb[0] = cr.e0p[0]; eb[1] = cr.e0p[1]; eb[2] = cr.e0p[2];
            }
        }
        const uint32_t sp = uni(zp < 0 ? 0u : (uint32_t)(zp * c.plane) << 2);
        bst3v(b.F1, (own2 && inp) ? c.o : OOB, sp, nb, eb);
        if (own2 && inp) {   // step n-1's gradient needs curl H^{n-1/2} - J^{n-1} and eps on the design box
            const long long di = box_index(c.x, c.y, zp, g.des_lo, g.des_hi);
            if (di >= 0) {
                const long long nd = (long long)(g.det_hi[0] - g.det_lo[0]) * (g.det_hi[1] - g.det_lo[1]) *
                                     (g.det_hi[2] - g.det_lo[2]);
                float* q = stash + 6 * nd + 4 * di;
                q[0] = u[0]; q[1] = u[1]; q[2] = u[2]; q[3] = cr.ep;
            }
        }
    }
    // ---- H^{n-3/2}(j-2) ----
    {
        const float ex = sEB[0][ly][lx], ey = sEB[1][ly][lx], ez = sEB[2][ly][lx];   // E^{n-1}(j-2), own
        float h[3];
        h[0] = cr.ha[0] + dt * ((sEB[2][ly + 1][lx] - ez) - (eb[1] - ey));
        h[1] = cr.ha[1] + dt * ((eb[0] - ex) - (sEB[2][ly][lx + 1] - ez));
        h[2] = cr.ha[2] + dt * ((sEB[1][ly][lx + 1] - ey) - (sEB[0][ly + 1][lx] - ex));
        const uint32_t sq = uni(zq < 0 ? 0u : (uint32_t)(zq * c.plane) << 2);
        bst3v(b.F1, (own3 && inq) ? c.o : OOB, sq + 3 * nb, nb, h);
    }
    sHin[0][ly][lx] = in.h[0];
    sHin[1][ly][lx] = in.h[1];
    sHin[2][ly][lx] = in.h[2];
    sEA[0][ly][lx] = ea[0];
    sEA[1][ly][lx] = ea[1];
    sEA[2][ly][lx] = ea[2];
    __syncthreads();   // B
    // ---- carry to iteration j+1 ----
    cr.h0p[0] = hx;
    cr.h0p[1] = hy;
    cr.h0p[2] = hz;
    #pragma unroll
    for (int q = 0; q < 3; ++q) { cr.e0p[q] = in.e[q]; cr.ha[q] = ha[q]; cr.eb[q] = eb[q]; }
    cr.ep = in.ep;
    cr.sp = in.sp;
}

// The march of one tile: the prologue (H^{n+1/2}(k0-2) of the own column, H^{n+1/2}(k0-1)
// into LDS, zero carries, the inputs of the first iteration), then iterations
// k0-1 .. k1+1, two per loop trip so that the inputs of iteration j+1 are loaded into the
// other register set before iteration j runs.
template <int HY, int CZ, bool FACES>
__device__ __forceinline__ void rev2_tile(const Grid& g, const Rev2Bufs& b, const Rev2Ctx& c, RPlane<HY>& sHin,
                                          RPlane<HY>& sEA, RPlane<HY>& sHA, RPlane<HY>& sEB,
                                          const ShellTile<HY, CZ>& st, float w0, float w1, float* __restrict__ Eb0,
                                          double* __restrict__ grad, float* __restrict__ stash) {
    RCarry cr;
    float hm[3];
    {
        const int zm = bound(c.k0 - 2, g.nz, g.periodic), z0 = bound(c.k0 - 1, g.nz, g.periodic);
        const uint32_t sm = uni(zm < 0 ? 0u : (uint32_t)(zm * c.plane) << 2);
        const uint32_t s0 = uni(z0 < 0 ? 0u : (uint32_t)(z0 * c.plane) << 2);
        bld3v(b.F0, zm < 0 ? OOB : c.f, sm + 3 * c.nb, c.nb, cr.h0p);
        bld3v(b.F0, z0 < 0 ? OOB : c.f, s0 + 3 * c.nb, c.nb, hm);
    }
    #pragma unroll
    for (int q = 0; q < 3; ++q) { cr.e0p[q] = 0.0f; cr.ha[q] = 0.0f; cr.eb[q] = 0.0f; }
    cr.ep = 1.0f;
    cr.sp = 0.0f;
    RIn pin[2];
    load_rin<HY, CZ>(g, b, c, c.k0 - 1, pin[0]);
    #pragma unroll
    for (int q = 0; q < 3; ++q) {
        sHin[q][c.row + 1][c.lane + 1] = hm[q];
        sEA[q][c.row + 1][c.lane + 1] = 0.0f;
    }
    __syncthreads();   // also publishes the shell tile
    const int cnt = c.k1 - c.k0 + 3;
    #pragma unroll 1
    for (int it = 0; it < cnt; it += 2) {
        const int j = c.k0 - 1 + it;
        if (it + 1 < cnt) load_rin<HY, CZ>(g, b, c, j + 1, pin[1]);
        iter_rev2<HY, CZ, FACES>(g, b, c, sHin, sEA, sHA, sEB, st, j, pin[0], cr, w0, w1, Eb0, grad, stash);
        if (it + 1 < cnt) {
            if (it + 2 < cnt) load_rin<HY, CZ>(g, b, c, j + 2, pin[0]);
            iter_rev2<HY, CZ, FACES>(g, b, c, sHin, sEA, sHA, sEB, st, j + 1, pin[1], cr, w0, w1, Eb0, grad, stash);
        }
    }
}

// Reverse steps n and n-1 on the interior: (E^{n+1}, H^{n+1/2}) in F0 -> (E^{n-1}, H^{n-3/2})
// in F1.  w0, w1: the source waveform at n and n-1.  Eb0: the adjoint fields of step n
// (E then H); grad: the FP64 gradient; stash: step n-1's seed and gradient inputs (the
// detector cells' E^n and H^{n-1/2}, then the design cells' curl H^{n-1/2} - J^{n-1} and
// eps); mid: step n's interface shell.
template <int HY, int CZ>
__global__ __launch_bounds__(TX * (HY + 4)) void k_rev2(Grid g, Tiling tl, const float* __restrict__ F0,
                                                        float* __restrict__ F1, const float* __restrict__ eps,
                                                        float* __restrict__ Eb0, float w0, float w1,
                                                        double* __restrict__ grad, float* __restrict__ stash,
                                                        const float* __restrict__ mid) {
    __shared__ RPlane<HY> sHin, sEA, sHA, sEB;
    __shared__ ShellTile<HY, CZ> st;
    const int P = g.P;
    const int Lt = logical_tile(tl);
    const int tix = Lt % tl.ntx, tiy = (Lt / tl.ntx) % tl.nty, tiz = Lt / (tl.ntx * tl.nty);
    const int a = P + tix * W2, j0 = P + tiy * HY;
    Rev2Ctx c;
    c.k0 = P + tiz * CZ;
    c.k1 = min(c.k0 + CZ, g.nz - P);
    c.lane = threadIdx.x;
    c.row = threadIdx.y;
    c.x = a - 2 + c.lane;
    c.y = j0 - 2 + c.row;
    c.plane = g.nx * g.ny;
    const int N = (int)g.N;
    c.nb = (uint32_t)N << 2;
    const Col col = make_col(g, c.x, c.y);
    c.live = col.xy >= 0;
    const bool ix = col.x >= P && col.x < g.nx - P, iy = col.y >= P && col.y < g.ny - P;
    c.inxy = c.live && ix && iy;
    c.own = c.lane >= 2 && c.lane < TX - 2 && c.row >= 2 && c.row < HY + 2 && c.x < g.nx - P && c.y < g.ny - P;
    c.xhe = P > 0 && c.live && col.x == g.nx - P && iy;
    c.xlh = P > 0 && c.live && col.x == P - 1 && iy;
    c.yhe = P > 0 && c.live && col.y == g.ny - P && ix;
    c.ylh = P > 0 && c.live && col.y == P - 1 && ix;
    c.f = lane_off(c.live, col.xy);
    c.o = lane_off(c.live && c.own, col.xy);
    const int sxn = g.src_hi[0] - g.src_lo[0], syn = g.src_hi[1] - g.src_lo[1];
    c.src = lane_off(c.live && col.x >= g.src_lo[0] && col.x < g.src_hi[0] && col.y >= g.src_lo[1] &&
                         col.y < g.src_hi[1],
                     (col.x - g.src_lo[0]) + sxn * (col.y - g.src_lo[1]));
    Rev2Bufs b;
    b.F0 = make_rsrc(F0, (uint32_t)(6 * N) * 4u);
    b.F1 = make_rsrc(F1, (uint32_t)(6 * N) * 4u);
    b.eps = make_rsrc(eps, (uint32_t)(c.plane * g.nz) * 4u);
    b.src = make_rsrc(g.src_profile, (uint32_t)(sxn * syn * (g.src_hi[2] - g.src_lo[2])) * 4u);
    // tiles whose cells all lie in I (planes k0-1 .. k1+1, two cells around in x and y)
    // need no shell
    const bool inner = a - 2 >= P && a + TX - 3 < g.nx - P && j0 - 2 >= P && j0 + HY + 1 < g.ny - P &&
                       c.k0 - 1 >= P && c.k1 + 1 < g.nz - P;
    if (inner) {
        rev2_tile<HY, CZ, false>(g, b, c, sHin, sEA, sHA, sEB, st, w0, w1, Eb0, grad, stash);
    } else {
        const int tid = c.row * TX + c.lane;
        if (P > 0) fill_shell_tile<HY, CZ>(g, st, mid, a, j0, c.k0, tid, TX * (HY + 4));   // published by the prologue's barrier
        rev2_tile<HY, CZ, true>(g, b, c, sHin, sEA, sHA, sEB, st, w0, w1, Eb0, grad, stash);
    }
}

// Step n-1's loss seed (added to the adjoint E, and H for a flux objective) and gradient
// term, after step n's transpose: one thread per detector cell outside the design box and
// per design cell (which takes its own seed first when it is also a detector cell), as
// the single-step reversal orders them.
__global__ __launch_bounds__(256) void k_rev_pending(Grid g, float* __restrict__ A, double* __restrict__ grad,
                                                     const float* __restrict__ stash, int ndet, int ndes) {
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= ndet + ndes) return;
    const long long N = g.N;
    const int dx = g.det_hi[0] - g.det_lo[0], dy = g.det_hi[1] - g.det_lo[1];
    auto seed = [&](int x, int y, int z, long long di, float eb[3]) {
        const float* q = stash + 6 * di;
        const float e[3] = {q[0], q[1], q[2]}, h[3] = {q[3], q[4], q[5]};
        float gE[3], gH[3];
        loss_seeds(g.loss, e, h, gE, gH);
        const long long idx = x + (long long)g.nx * (y + (long long)g.ny * z);
        eb[0] = A[idx] + gE[0];
        eb[1] = A[N + idx] + gE[1];
        eb[2] = A[2 * N + idx] + gE[2];
        A[idx] = eb[0];
        A[N + idx] = eb[1];
        A[2 * N + idx] = eb[2];
        if (g.loss != 0) {
            A[3 * N + idx] += gH[0];
            A[4 * N + idx] += gH[1];
            A[5 * N + idx] += gH[2];
        }
    };
    if (t < ndet) {
        const int x = g.det_lo[0] + t % dx, y = g.det_lo[1] + (t / dx) % dy, z = g.det_lo[2] + t / (dx * dy);
        if (in_box(x, y, z, g.des_lo, g.des_hi)) return;   // the design thread takes it
        float eb[3];
        seed(x, y, z, t, eb);
        return;
    }
    const int d = t - ndet;
    const int ex = g.des_hi[0] - g.des_lo[0], ey = g.des_hi[1] - g.des_lo[1];
    const int x = g.des_lo[0] + d % ex, y = g.des_lo[1] + (d / ex) % ey, z = g.des_lo[2] + d / (ex * ey);
    float eb[3];
    const long long di = box_index(x, y, z, g.det_lo, g.det_hi);
    if (di >= 0) {
        seed(x, y, z, di, eb);
    } else {
        const long long idx = x + (long long)g.nx * (y + (long long)g.ny * z);
        eb[0] = A[idx];
        eb[1] = A[N + idx];
        eb[2] = A[2 * N + idx];
    }
    const float* q = stash + 6LL * ndet + 4LL * d;
    const double ee = (double)q[3];
    const double s = (double)eb[0] * q[0] + (double)eb[1] * q[1] + (double)eb[2] * q[2];
    grad[d] -= (double)g.dt / (ee * ee) * s;
}

template <int HY, int CZ>
static void launch_rev2_t(const Grid& g, const Tiling& t, const float* F0, float* F1, const float* eps, float* Eb0,
                          float w0, float w1, double* grad, float* stash, const float* mid, hipStream_t s) {
    launch_kernel(K_PRIM_REV2, k_rev2<HY, CZ>, dim3(t.count), dim3(TX, HY + 4), s, g, t, F0, F1, eps, Eb0, w0, w1,
                  grad, stash, mid);
}

void launch_rev2(const Grid& g, const Tiling& t, const float* F0, float* F1, const float* eps, float* Eb0,
                 float wave_n, float wave_n1, double* grad, float* stash, const float* mid, hipStream_t s) {
    if (t.cz == 8) launch_rev2_t<12, 8>(g, t, F0, F1, eps, Eb0, wave_n, wave_n1, grad, stash, mid, s);
    else launch_rev2_t<12, 16>(g, t, F0, F1, eps, Eb0, wave_n, wave_n1, grad, stash, mid, s);
}

void launch_rev_pending(const Grid& g, float* A, double* grad, const float* stash, hipStream_t s) {
    const int ndet = (g.det_hi[0] - g.det_lo[0]) * (g.det_hi[1] - g.det_lo[1]) * (g.det_hi[2] - g.det_lo[2]);
    const int ndes = (g.des_hi[0] - g.des_lo[0]) * (g.des_hi[1] - g.des_lo[1]) * (g.des_hi[2] - g.des_lo[2]);
    const int n = ndet + ndes;
    launch_kernel(K_REV_PENDING, k_rev_pending, dim3((unsigned)((n + 255) / 256)), dim3(256), s, g, A, grad, stash,
                  ndet, ndes);
}

}  // namespace fdtd
