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

}  // namespace fdtd
