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
constexpr int W2 = TX - 4;    // owned columns of a two-step forward tile (two halo cells each side)

struct Tiling {
    int ty;                   // rows per tile (threads in y)
    int cz;                   // planes per block
    int ntx, nty, ntz;        // tiles per axis
    int count;                // blocks
    // tiles intersecting the detector box (loss partials)
    int dtx0, dty0, dtz0, dntx, dnty, dntz;
    // launch order of the tiles (count entries, device), or NULL for x-y-z order: tiles
    // grouped by class, so that the blocks one compute unit runs at a time mostly share
    // one of the class-specialised code paths (one path fills much of the instruction
    // cache; blocks of several classes side by side had evicted each other's code)
    const int32_t* order;
};

// The tile of this block: workgroups go to the 8 XCDs round-robin, so position
// (w & 7) * per + (w >> 3) gives each XCD one contiguous range of the order.
__device__ inline int logical_tile(const Tiling& t) {
    const int w = blockIdx.x;
    const int per = t.count >> 3;
    const int full = per << 3;
    const int p = w < full ? (w & 7) * per + (w >> 3) : w;
    return t.order ? t.order[p] : p;
}

// Index along an axis after the boundary rule: -1 means "outside, value 0".
__device__ inline int bound(int x, int n, int periodic) {
    if (x >= 0 && x < n) return x;
    if (!periodic) return -1;
    return x < 0 ? x + n : x - n;
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
// sx + 2P y, y slab x + nx sy, z slab x + nx y, 8 bytes per cell (the pair of one axis
// and side), OOB outside the slab or when off.
struct PsiLane {
    uint32_t x, y, z;
};
__device__ inline uint32_t lane_off8(bool on, int idx) { return on ? (uint32_t)idx << 3 : OOB; }
__device__ inline PsiLane psi_lane(const Grid& g, const Col& c, bool on) {
    PsiLane l;
    l.x = lane_off8(on && c.sx >= 0, c.sx + 2 * g.P * c.y);
    l.y = lane_off8(on && c.sy >= 0, c.x + g.nx * c.sy);
    l.z = lane_off8(on && c.xy >= 0 && g.P > 0, c.xy);
    return l;
}
// Plane-uniform part for one side (0 H, 1 E) on plane z of the copy at byte offset `base`.
struct PsiPlane {
    uint32_t x, y, z;
    bool zs;                  // plane z lies in a z slab
};
__device__ inline PsiPlane psi_plane(const Grid& g, int side, int z, uint32_t base) {
    PsiPlane p;
    const int P = g.P;
    const int sz = P > 0 ? slab_coord(z, g.nz, P) : -1;
    p.zs = sz >= 0;
    p.x = uni(base + ((uint32_t)(g.psi_off[0] + side * 2 * g.slab[0]) << 2) + ((uint32_t)(2LL * P * g.ny * z) << 3));
    p.y = uni(base + ((uint32_t)(g.psi_off[1] + side * 2 * g.slab[1]) << 2) + ((uint32_t)(2LL * P * g.nx * z) << 3));
    p.z = uni(base + ((uint32_t)(g.psi_off[2] + side * 2 * g.slab[2]) << 2) +
              ((uint32_t)((long long)g.nx * g.ny * (p.zs ? sz : 0)) << 3));
    return p;
}
// The two auxiliaries of one axis and side at one cell, in one 64-bit access.
typedef uint32_t u32x2 __attribute__((vector_size(8)));   // the type the 64-bit buffer builtins take and return
__device__ inline void bld2v(rsrc_t r, uint32_t v, uint32_t s, float& a, float& b) {
    const u32x2 u = __builtin_amdgcn_raw_buffer_load_b64(r, v, s, FDTD_LD_AUX);
    // each element through a scalar first: a bit cast of a vector element in place
    // reads the vector's first element
    const uint32_t lo = u[0], hi = u[1];
    a = __builtin_bit_cast(float, lo);
    b = __builtin_bit_cast(float, hi);
}
__device__ inline void bst2v(rsrc_t r, uint32_t v, uint32_t s, float a, float b) {
    u32x2 u;
    u[0] = __builtin_bit_cast(uint32_t, a);
    u[1] = __builtin_bit_cast(uint32_t, b);
    __builtin_amdgcn_raw_buffer_store_b64(u, r, v, s, FDTD_ST_AUX);
}
// The six auxiliaries (x: 3, 4; y: 0, 5; z: 1, 2) of the axes whose slabs a tile of
// class SL (bit 0: x, 1: y, 2: z) reaches; out-of-slab cells read 0 and their stores are
// dropped.  The other axes' auxiliaries are neither loaded nor stored (they would be
// out of range for every cell of the tile) and read as 0.
template <int SL>
__device__ inline void bld_psi_s(rsrc_t r, const PsiLane& l, const PsiPlane& p, float v[6]) {
    v[0] = v[1] = v[2] = v[3] = v[4] = v[5] = 0.0f;
    if constexpr ((SL & 1) != 0) bld2v(r, l.x, p.x, v[3], v[4]);
    if constexpr ((SL & 2) != 0) bld2v(r, l.y, p.y, v[0], v[5]);
    if constexpr ((SL & 4) != 0) bld2v(r, p.zs ? l.z : OOB, p.z, v[1], v[2]);
}
template <int SL>
__device__ inline void bst_psi_s(rsrc_t r, const PsiLane& l, const PsiPlane& p, const float v[6]) {
    if constexpr ((SL & 1) != 0) bst2v(r, l.x, p.x, v[3], v[4]);
    if constexpr ((SL & 2) != 0) bst2v(r, l.y, p.y, v[0], v[5]);
    if constexpr ((SL & 4) != 0) bst2v(r, p.zs ? l.z : OOB, p.z, v[1], v[2]);
}

// Class of a tile: which axes' PML slabs (bit 0: x, 1: y, 2: z) reach the cells
// [x0, x1] x [y0, y1] x [z0, z1] it touches (ranges clipped to the grid).  Outside a
// slab of its axis the coefficients are (0, 0, 1), so skipping an axis that no cell of
// the tile lies in changes no value.
__host__ __device__ inline int slab_class(const Grid& g, int x0, int x1, int y0, int y1, int z0, int z1) {
    if (g.P == 0) return 0;
    auto reaches = [&](int lo, int hi, int n) {
        lo = lo < 0 ? 0 : lo;
        hi = hi > n - 1 ? n - 1 : hi;
        return lo <= hi && (lo < g.P || hi >= n - g.P);
    };
    return (reaches(x0, x1, g.nx) ? 1 : 0) | (reaches(y0, y1, g.ny) ? 2 : 0) | (reaches(z0, z1, g.nz) ? 4 : 0);
}

// CPML of one axis on its two terms: psi <- b psi + a t, t <- kinv t + psi; the y and z parts run under
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
// CPML on the six differences t of one half step, on the axes of tile class SL
template <int SL>
__device__ inline void cpml_axes(const Cf& cx, const Cf& cy, const Cf& cz, float t[6], float p[6]) {
    if constexpr ((SL & 1) != 0) cpml_x(cx, t, p);
    if constexpr ((SL & 2) != 0) cpml_y(cy, t, p);
    if constexpr ((SL & 4) != 0) cpml_z(cz, t, p);
}

}  // namespace fdtd
