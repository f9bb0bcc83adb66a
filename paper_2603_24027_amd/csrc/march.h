// Tiling shared by the fused sweeps: 2.5-D z-marching blocks with LDS planes.
//
// A block owns a tile of TX x TY cells in (x, y) (one wavefront per row of 64
// cells) and marches over CZ consecutive z-planes.  The two halves of a
// leapfrog step are fused: the first half is evaluated on the tile plus a
// one-cell halo on the side the second half reads, from an LDS copy of the
// input plane that carries its own one-cell halo ring; the second half then
// reads the first half's results from LDS (x, y neighbours) and registers
// (the previous plane).  Inputs are read from one buffer and outputs written
// to the other (ping-pong), so a halo value recomputed by a neighbouring
// block always sees the same old inputs as its owner.
//
// Blocks are numbered so that each XCD (the hardware hands workgroups to the
// 8 XCDs round-robin) receives one contiguous range of tiles in x-y-z order:
// tiles that share halo cache lines then share that XCD's L2.
#pragma once

#include "common.h"

namespace fdtd {

constexpr int TX = 64;        // cells per tile row (one wavefront)
constexpr int EXT = TX + 2;   // LDS row length: tile plus a halo column on each side

struct Tiling {
    int ty;                   // rows per tile (threads in y)
    int cz;                   // planes per block
    int ntx, nty, ntz;        // tiles per axis
    int count;                // blocks
    // tiles intersecting the detector box (loss partials)
    int dtx0, dty0, dtz0, dntx, dnty, dntz;
};

__device__ inline int logical_tile(int count) {
    const int w = blockIdx.x;
    const int per = count >> 3;
    const int full = per << 3;
    return w < full ? (w & 7) * per + (w >> 3) : w;
}

// Index along an axis after the boundary rule: -1 means "outside, value 0".
__device__ inline int bound(int x, int n, int periodic) {
    if (x >= 0 && x < n) return x;
    if (!periodic) return -1;
    return x < 0 ? x + n : x - n;
}

__device__ inline float ldg(const float* f, const Grid& g, int x, int y, int z) {
    const int bx = bound(x, g.nx, g.periodic), by = bound(y, g.ny, g.periodic), bz = bound(z, g.nz, g.periodic);
    if ((bx | by | bz) < 0) return 0.0f;
    return f[bx + g.nx * (by + g.ny * bz)];
}

// Load plane z of the three components of a field into the extended LDS plane
// s[c][ly][lx] (ly in [0, TY+2), lx in [0, EXT)), covering x in [i0-1, i0+TX],
// y in [j0-1, j0+TY].  Every cell, inside the domain or not, receives the value
// the boundary rule gives it.
template <int TY>
__device__ inline void load_ext_plane(float (*s)[TY + 2][EXT], const float* f, int N, const Grid& g,
                                      int i0, int j0, int z) {
    const int lane = threadIdx.x, ty = threadIdx.y;
    #pragma unroll
    for (int c = 0; c < 3; ++c) s[c][ty + 1][lane + 1] = ldg(f + c * N, g, i0 + lane, j0 + ty, z);
    if (ty == 0) {
        #pragma unroll
        for (int c = 0; c < 3; ++c) s[c][0][lane + 1] = ldg(f + c * N, g, i0 + lane, j0 - 1, z);
    } else if (ty == 1) {
        #pragma unroll
        for (int c = 0; c < 3; ++c) s[c][TY + 1][lane + 1] = ldg(f + c * N, g, i0 + lane, j0 + TY, z);
    } else if (ty == 2 && lane < TY + 2) {
        #pragma unroll
        for (int c = 0; c < 3; ++c) s[c][lane][0] = ldg(f + c * N, g, i0 - 1, j0 - 1 + lane, z);
    } else if (ty == 3 && lane < TY + 2) {
        #pragma unroll
        for (int c = 0; c < 3; ++c) s[c][lane][EXT - 1] = ldg(f + c * N, g, i0 + TX, j0 - 1 + lane, z);
    }
}

// A column (x, y) of the grid after the boundary rule, with what a sweep needs
// to address it on any plane: xy = x + nx y (or -1: outside, value 0) and the
// slab coordinates along x and y (-1 outside the slab).
struct Col {
    int xy;
    int x, y;
    int sx, sy;
};

__device__ inline Col make_col(const Grid& g, int xr, int yr) {
    Col c;
    c.x = bound(xr, g.nx, g.periodic);
    c.y = bound(yr, g.ny, g.periodic);
    c.xy = (c.x >= 0 && c.y >= 0) ? c.x + g.nx * c.y : -1;
    c.sx = (c.xy >= 0 && g.P > 0) ? slab_coord(c.x, g.nx, g.P) : -1;
    c.sy = (c.xy >= 0 && g.P > 0) ? slab_coord(c.y, g.ny, g.P) : -1;
    return c;
}

// Per-block state of a forward-shaped sweep (forward step, adjoint step) that does
// not change along z: the own column, the LDS-ring position this thread loads
// (rlx, rly; -1 if none) and the first-half halo cell it evaluates (hex, hey).
template <int TY>
struct FwdCtx {
    int i0, j0, lane, row, tid, x, y, N, P, plane;
    bool live;
    Col own, ring, hc;
    int rlx, rly, hex, hey;
};

__device__ inline void load3(const float* __restrict__ f, int N, int idx, float v[3]) {
    if (idx < 0) { v[0] = v[1] = v[2] = 0.0f; return; }
    v[0] = f[idx];
    v[1] = f[N + idx];
    v[2] = f[2 * N + idx];
}

// Offsets of the two auxiliaries of each axis slab of a cell on plane z
// (slab coordinate along z: sz): o[0] x-slab, o[1] y-slab, o[2] z-slab, -1 if
// the cell is not in that slab.  side 0 = H-half arrays, 1 = E-half arrays.
__device__ inline void psi_offsets(const Grid& g, const Col& c, int z, int sz, int side, int o[3]) {
    const int P = g.P;
    o[0] = c.sx >= 0 ? (int)(g.psi_off[0] + side * 2 * g.slab[0]) + c.sx + 2 * P * (c.y + g.ny * z) : -1;
    o[1] = c.sy >= 0 ? (int)(g.psi_off[1] + side * 2 * g.slab[1]) + c.x + g.nx * (c.sy + 2 * P * z) : -1;
    o[2] = (sz >= 0 && c.xy >= 0) ? (int)(g.psi_off[2] + side * 2 * g.slab[2]) + c.x + g.nx * (c.y + g.ny * sz) : -1;
}

// Auxiliaries of the six terms (x: 3, 4; y: 0, 5; z: 1, 2) at those offsets; 0 outside the slabs.
__device__ inline void load_psi(const Grid& g, const float* __restrict__ psi, const int o[3], float p[6]) {
    p[0] = p[1] = p[2] = p[3] = p[4] = p[5] = 0.0f;
    if (o[0] >= 0) { p[3] = psi[o[0]]; p[4] = psi[o[0] + (int)g.slab[0]]; }
    if (o[1] >= 0) { p[0] = psi[o[1]]; p[5] = psi[o[1] + (int)g.slab[1]]; }
    if (o[2] >= 0) { p[1] = psi[o[2]]; p[2] = psi[o[2] + (int)g.slab[2]]; }
}

__device__ inline void store_psi(const Grid& g, float* __restrict__ psi, const int o[3], const float p[6]) {
    if (o[0] >= 0) { psi[o[0]] = p[3]; psi[o[0] + (int)g.slab[0]] = p[4]; }
    if (o[1] >= 0) { psi[o[1]] = p[0]; psi[o[1] + (int)g.slab[1]] = p[5]; }
    if (o[2] >= 0) { psi[o[2]] = p[1]; psi[o[2] + (int)g.slab[2]] = p[2]; }
}

// CPML on the six differences t of one half step: inside the slab of a term's
// axis, psi <- b psi + a t and t <- kinv t + psi (table: b | a | kinv, 2P each).
__device__ inline void cpml_terms(const float* __restrict__ tab, int P, const Col& c, int sz, float t[6],
                                  float p[6]) {
    if (P == 0) return;
    const float* b = tab;
    const float* a = tab + 2 * P;
    const float* kv = tab + 4 * P;
    if (c.sx >= 0) {
        const int s = c.sx;
        p[3] = b[s] * p[3] + a[s] * t[3]; t[3] = kv[s] * t[3] + p[3];
        p[4] = b[s] * p[4] + a[s] * t[4]; t[4] = kv[s] * t[4] + p[4];
    }
    if (c.sy >= 0) {
        const int s = c.sy;
        p[0] = b[s] * p[0] + a[s] * t[0]; t[0] = kv[s] * t[0] + p[0];
        p[5] = b[s] * p[5] + a[s] * t[5]; t[5] = kv[s] * t[5] + p[5];
    }
    if (sz >= 0) {
        const int s = sz;
        p[1] = b[s] * p[1] + a[s] * t[1]; t[1] = kv[s] * t[1] + p[1];
        p[2] = b[s] * p[2] + a[s] * t[2]; t[2] = kv[s] * t[2] + p[2];
    }
}

// ---------------------------------------------------------------------------
// Range-checked buffer access.  A load at an offset past the buffer returns 0
// and a store there is dropped (raw buffer resource, stride 0), so a sweep can
// read "outside the domain" and skip the writes of idle lanes without a branch:
// its loads and stores then form straight-line code and the compiler waits for
// exactly the values it needs.
// ---------------------------------------------------------------------------
using rsrc_t = __amdgpu_buffer_rsrc_t;
// cache-policy bits of the sweeps' buffer loads and stores (a translation unit
// may set them before including this header); non-temporal hints (bit 1) were
// measured 15-20 % slower on every sweep
#ifndef FDTD_LD_AUX
#define FDTD_LD_AUX 0
#endif
#ifndef FDTD_ST_AUX
#define FDTD_ST_AUX 0
#endif
constexpr uint32_t OOB = 0x80000000u;          // every buffer here is smaller than 2 GiB

__device__ inline rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline float bld(rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, FDTD_LD_AUX));
}
__device__ inline void bst(rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, FDTD_ST_AUX);
}
// byte offset of element idx of component c of a 3-component field (OOB when idx < 0)
__device__ inline uint32_t foff(int idx, int c, int N) {
    return idx < 0 ? OOB : (uint32_t)(idx + c * N) << 2;
}
__device__ inline void bld3(rsrc_t r, int idx, int N, float v[3]) {
    v[0] = bld(r, foff(idx, 0, N));
    v[1] = bld(r, foff(idx, 1, N));
    v[2] = bld(r, foff(idx, 2, N));
}
__device__ inline void bst3(rsrc_t r, int idx, int N, const float v[3]) {
    bst(r, foff(idx, 0, N), v[0]);
    bst(r, foff(idx, 1, N), v[1]);
    bst(r, foff(idx, 2, N), v[2]);
}
// PML auxiliaries of the six terms at the offsets of psi_offsets (x: 3, 4; y: 0, 5; z: 1, 2)
__device__ inline void bld_psi(const Grid& g, rsrc_t r, const int o[3], float p[6]) {
    const uint32_t ox = o[0] < 0 ? OOB : (uint32_t)o[0] << 2, oy = o[1] < 0 ? OOB : (uint32_t)o[1] << 2;
    const uint32_t oz = o[2] < 0 ? OOB : (uint32_t)o[2] << 2;
    p[3] = bld(r, ox); p[4] = bld(r, ox == OOB ? OOB : ox + ((uint32_t)g.slab[0] << 2));
    p[0] = bld(r, oy); p[5] = bld(r, oy == OOB ? OOB : oy + ((uint32_t)g.slab[1] << 2));
    p[1] = bld(r, oz); p[2] = bld(r, oz == OOB ? OOB : oz + ((uint32_t)g.slab[2] << 2));
}
__device__ inline void bst_psi(const Grid& g, rsrc_t r, const int o[3], const float p[6]) {
    const uint32_t ox = o[0] < 0 ? OOB : (uint32_t)o[0] << 2, oy = o[1] < 0 ? OOB : (uint32_t)o[1] << 2;
    const uint32_t oz = o[2] < 0 ? OOB : (uint32_t)o[2] << 2;
    bst(r, ox, p[3]); bst(r, ox == OOB ? OOB : ox + ((uint32_t)g.slab[0] << 2), p[4]);
    bst(r, oy, p[0]); bst(r, oy == OOB ? OOB : oy + ((uint32_t)g.slab[1] << 2), p[5]);
    bst(r, oz, p[1]); bst(r, oz == OOB ? OOB : oz + ((uint32_t)g.slab[2] << 2), p[2]);
}

// CPML coefficients of one axis at one position: psi <- b psi + a t, t <- kinv t + psi.
// Outside the axis slab the triple is (0, 0, 1), which leaves t unchanged and psi 0,
// so the update needs no branch.
struct Cf {
    float b, a, k;
};

// Per-block LDS copy of the coefficients along each axis of a tile with a one-cell
// halo ring and its CZ planes plus one on each side (z = k0-1 .. k0+CZ):
// [side 0 E / 1 H][b | a | kinv][position].
template <int TY, int CZ>
struct CoefTile {
    float x[2][3][EXT];
    float y[2][3][TY + 2];
    float z[2][3][CZ + 2];
};

__device__ inline float coef_at(const Grid& g, int side, int kind, int pos, int n) {
    const int b = bound(pos, n, g.periodic);
    const int s = (b >= 0 && g.P > 0) ? slab_coord(b, n, g.P) : -1;
    if (s < 0) return kind == 2 ? 1.0f : 0.0f;
    return g.coef[6 * g.P * side + 2 * g.P * kind + s];
}

// Fill the tile's coefficient table (all threads of the block; a barrier follows).
template <int TY, int CZ>
__device__ inline void fill_coef_tile(const Grid& g, CoefTile<TY, CZ>& ct, int i0, int j0, int k0, int tid,
                                      int nthreads) {
    constexpr int NX = 6 * EXT, NY = 6 * (TY + 2), NZ = 6 * (CZ + 2);
    for (int e = tid; e < NX + NY + NZ; e += nthreads) {
        if (e < NX) {
            const int side = e / (3 * EXT), kind = (e / EXT) % 3, pos = e % EXT;
            ct.x[side][kind][pos] = coef_at(g, side, kind, i0 - 1 + pos, g.nx);
        } else if (e < NX + NY) {
            const int r = e - NX, side = r / (3 * (TY + 2)), kind = (r / (TY + 2)) % 3, pos = r % (TY + 2);
            ct.y[side][kind][pos] = coef_at(g, side, kind, j0 - 1 + pos, g.ny);
        } else {
            const int r = e - NX - NY, side = r / (3 * (CZ + 2)), kind = (r / (CZ + 2)) % 3, pos = r % (CZ + 2);
            ct.z[side][kind][pos] = coef_at(g, side, kind, k0 - 1 + pos, g.nz);
        }
    }
}

template <int TY, int CZ>
__device__ inline Cf cf_x(const CoefTile<TY, CZ>& ct, int side, int lx) {
    return Cf{ct.x[side][0][lx], ct.x[side][1][lx], ct.x[side][2][lx]};
}
template <int TY, int CZ>
__device__ inline Cf cf_y(const CoefTile<TY, CZ>& ct, int side, int ly) {
    return Cf{ct.y[side][0][ly], ct.y[side][1][ly], ct.y[side][2][ly]};
}
template <int TY, int CZ>
__device__ inline Cf cf_z(const CoefTile<TY, CZ>& ct, int side, int lz) {
    return Cf{ct.z[side][0][lz], ct.z[side][1][lz], ct.z[side][2][lz]};
}

// Branch-free CPML on the six differences t of one half step (x: 3, 4; y: 0, 5; z: 1, 2).
__device__ inline void cpml_apply(const Cf& cx, const Cf& cy, const Cf& cz, float t[6], float p[6]) {
    p[3] = cx.b * p[3] + cx.a * t[3]; t[3] = cx.k * t[3] + p[3];
    p[4] = cx.b * p[4] + cx.a * t[4]; t[4] = cx.k * t[4] + p[4];
    p[0] = cy.b * p[0] + cy.a * t[0]; t[0] = cy.k * t[0] + p[0];
    p[5] = cy.b * p[5] + cy.a * t[5]; t[5] = cy.k * t[5] + p[5];
    p[1] = cz.b * p[1] + cz.a * t[1]; t[1] = cz.k * t[1] + p[1];
    p[2] = cz.b * p[2] + cz.a * t[2]; t[2] = cz.k * t[2] + p[2];
}

// Loads and stores addressed as a per-lane byte offset v (loop-invariant: the
// lane's column, or OOB) plus a wave-uniform byte offset s (plane, component),
// so that the z-march spends no vector instructions on addresses.  An OOB lane
// offset stays out of range whatever s is added (every buffer is below 2 GiB).
__device__ inline float bldv(rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, FDTD_LD_AUX));
}
__device__ inline void bstv(rsrc_t r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, v, s, FDTD_ST_AUX);
}
// three components of a field: component c at s + c * nb (nb = 4 N)
__device__ inline void bld3v(rsrc_t r, uint32_t v, uint32_t s, uint32_t nb, float o[3]) {
    o[0] = bldv(r, v, s);
    o[1] = bldv(r, v, s + nb);
    o[2] = bldv(r, v, s + 2 * nb);
}
__device__ inline void bst3v(rsrc_t r, uint32_t v, uint32_t s, uint32_t nb, const float o[3]) {
    bstv(r, v, s, o[0]);
    bstv(r, v, s + nb, o[1]);
    bstv(r, v, s + 2 * nb, o[2]);
}
__device__ inline uint32_t lane_off(bool on, int idx) { return on ? (uint32_t)idx << 2 : OOB; }

// Offsets into a [z][y][x] profile over the box [lo, hi): the lane part for column c
// (OOB outside the box in x-y) and the plane part for plane z (false outside in z).
__device__ inline uint32_t box_lane(const int lo[3], const int hi[3], const Col& c) {
    const bool in = c.xy >= 0 && c.x >= lo[0] && c.x < hi[0] && c.y >= lo[1] && c.y < hi[1];
    return lane_off(in, (c.x - lo[0]) + (hi[0] - lo[0]) * (c.y - lo[1]));
}
__device__ inline bool box_plane(const int lo[3], const int hi[3], int z, uint32_t& s);
// a value the caller knows to be wave-uniform, kept in a scalar register (the buffer
// instructions take their uniform offset from one)
__device__ inline uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

__device__ inline bool box_plane(const int lo[3], const int hi[3], int z, uint32_t& s) {
    const bool in = z >= lo[2] && z < hi[2];
    s = uni(in ? (uint32_t)((z - lo[2]) * (hi[0] - lo[0]) * (hi[1] - lo[1])) << 2 : 0u);
    return in;
}

// Per-lane part of the byte offsets of a column's PML auxiliaries: x slab
// sx + 2P y, y slab x + nx sy, z slab x + nx y (OOB outside the slab or when off).
struct PsiLane {
    uint32_t x, y, z;
};
__device__ inline PsiLane psi_lane(const Grid& g, const Col& c, bool on) {
    PsiLane l;
    l.x = lane_off(on && c.sx >= 0, c.sx + 2 * g.P * c.y);
    l.y = lane_off(on && c.sy >= 0, c.x + g.nx * c.sy);
    l.z = lane_off(on && c.xy >= 0 && g.P > 0, c.xy);
    return l;
}
// Plane-uniform part for one side (0 H, 1 E) on plane z of the copy at byte offset
// `base`, and the distance to the second auxiliary of each slab.
struct PsiPlane {
    uint32_t x, y, z, dx, dy, dz;
    bool zs;                  // plane z lies in a z slab
};
__device__ inline PsiPlane psi_plane(const Grid& g, int side, int z, uint32_t base) {
    PsiPlane p;
    const int P = g.P;
    const int sz = P > 0 ? slab_coord(z, g.nz, P) : -1;
    p.zs = sz >= 0;
    p.x = uni(base + ((uint32_t)(g.psi_off[0] + side * 2 * g.slab[0] + 2LL * P * g.ny * z) << 2));
    p.y = uni(base + ((uint32_t)(g.psi_off[1] + side * 2 * g.slab[1] + 2LL * P * g.nx * z) << 2));
    p.z = uni(base + ((uint32_t)(g.psi_off[2] + side * 2 * g.slab[2] + (long long)g.nx * g.ny * (p.zs ? sz : 0)) << 2));
    p.dx = (uint32_t)g.slab[0] << 2;
    p.dy = (uint32_t)g.slab[1] << 2;
    p.dz = (uint32_t)g.slab[2] << 2;
    return p;
}
// the six auxiliaries (x: 3, 4; y: 0, 5; z: 1, 2); 0 outside the slabs
__device__ inline void bld_psi_v(rsrc_t r, const PsiLane& l, const PsiPlane& p, float v[6]) {
    const uint32_t vz = p.zs ? l.z : OOB;
    v[3] = bldv(r, l.x, p.x); v[4] = bldv(r, l.x, p.x + p.dx);
    v[0] = bldv(r, l.y, p.y); v[5] = bldv(r, l.y, p.y + p.dy);
    v[1] = bldv(r, vz, p.z); v[2] = bldv(r, vz, p.z + p.dz);
}
__device__ inline void bst_psi_v(rsrc_t r, const PsiLane& l, const PsiPlane& p, const float v[6]) {
    const uint32_t vz = p.zs ? l.z : OOB;
    bstv(r, l.x, p.x, v[3]); bstv(r, l.x, p.x + p.dx, v[4]);
    bstv(r, l.y, p.y, v[0]); bstv(r, l.y, p.y + p.dy, v[5]);
    bstv(r, vz, p.z, v[1]); bstv(r, vz, p.z + p.dz, v[2]);
}

// CPML of one axis on its two terms (see cpml_apply); the y and z parts run under
// wave-uniform branches, the x part (which varies across a wave) always.
__device__ inline void cpml_x(const Cf& c, float t[6], float p[6]) {
    p[3] = c.b * p[3] + c.a * t[3]; t[3] = c.k * t[3] + p[3];
    p[4] = c.b * p[4] + c.a * t[4]; t[4] = c.k * t[4] + p[4];
}
__device__ inline void cpml_y(const Cf& c, float t[6], float p[6]) {
    p[0] = c.b * p[0] + c.a * t[0]; t[0] = c.k * t[0] + p[0];
    p[5] = c.b * p[5] + c.a * t[5]; t[5] = c.k * t[5] + p[5];
}
__device__ inline void cpml_z(const Cf& c, float t[6], float p[6]) {
    p[1] = c.b * p[1] + c.a * t[1]; t[1] = c.k * t[1] + p[1];
    p[2] = c.b * p[2] + c.a * t[2]; t[2] = c.k * t[2] + p[2];
}

}  // namespace fdtd
