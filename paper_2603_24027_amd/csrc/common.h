// Shared device-side definitions of the FDTD gradient library (gfx950).
//
// Grid arrays are float32 structure-of-arrays, x fastest; the six field
// components of one buffer are [Ex | Ey | Ez | Hx | Hy | Hz], N cells each.
//
// Curl terms, numbered t = 0..5 for both halves of a step
// (component c, axis d, sign s, source field f):
//   H half (curl E, forward differences):
//     0 (Hx, y, +, Ez)  1 (Hx, z, -, Ey)  2 (Hy, z, +, Ex)
//     3 (Hy, x, -, Ez)  4 (Hz, x, +, Ey)  5 (Hz, y, -, Ex)
//   E half (curl H, backward differences):
//     0 (Ex, y, +, Hz)  1 (Ex, z, -, Hy)  2 (Ey, z, +, Hx)
//     3 (Ey, x, -, Hz)  4 (Ez, x, +, Hy)  5 (Ez, y, -, Hx)
// so axis x carries terms 3 and 4, axis y terms 0 and 5, axis z terms 1 and 2.
//
// Convolutional-PML auxiliaries live only in the slabs [0, P) and [n-P, n) of
// their axis.  Slab of axis d, slab coordinate i' in [0, 2P):
//   i' = i for i < P, i' = i - (n - 2P) for i >= n - P.
// Within the PML buffer each axis owns two arrays of slab-sized cell pairs,
//   [H (term a, term b) | E (term a, term b)] with (a, b) = (3, 4) for x,
//   (0, 5) for y and (1, 2) for z, the two terms of a cell adjacent (one 64-bit
//   access);  slab cell order (x fastest):
//   x: i' + 2P (j + ny k),  y: i + nx (j' + 2P k),  z: i + nx (j + ny k').
// The CPML coefficients depend on i' only (same thickness on every face),
// so one table of 2P entries per node type serves all three axes:
//   coef = [bE | aE | kinvE | bH | aH | kinvH], 2P floats each.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdtd {

constexpr int BX = 64;   // threads along x (one wavefront per x segment)
constexpr int BY = 4;    // rows per block

struct Grid {
    int nx, ny, nz, P;
    int periodic;
    int mx, my, mz;          // interior extents n - 2P
    long long N;             // floats between field components (>= cells)
    float dt;
    long long psi_off[3];    // start of each axis' four slab arrays in a PML buffer (floats)
    long long slab[3];       // slab size per axis (floats)
    long long psi_total;     // floats in one PML buffer
    const float* coef;       // device coefficient table (6 * 2P floats)
    // source
    int loss;                // 0: |E|^2 on the detector; 1, 2, 3: Poynting flux along x, y, z
    int msrc_comp;           // magnetic current sheet (empty box: none)
    int msrc_lo[3], msrc_hi[3];
    const float* msrc_profile;
    int src_comp;
    int src_lo[3], src_hi[3];
    const float* src_profile;
    // detector and design boxes
    int det_lo[3], det_hi[3];
    int des_lo[3], des_hi[3];
    // interface store
    int dtype;
    long long vps;           // values per kept step
    long long slice_stride;  // bytes between kept steps in the store
    long long scale_off;     // byte offset of the FP8 scale table in the store
    // detector-loss partials (forward): blocks intersecting the detector
    int dbx0, dby0, dbz0, dnbx, dnby, dnbz;
};

// ----------------------------------------------------------------------------
// Codec (bit-width reduction of recorded values).  All encoders round to
// nearest, ties to even, as the IEEE default.
// ----------------------------------------------------------------------------

__host__ __device__ inline uint32_t f2u(float x) {
    union { float f; uint32_t u; } v; v.f = x; return v.u;
}
__host__ __device__ inline float u2f(uint32_t u) {
    union { float f; uint32_t u; } v; v.u = u; return v.f;
}

__host__ __device__ inline uint16_t enc_bf16(float x) {
    uint32_t u = f2u(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);   // quiet NaN
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7fffu + lsb) >> 16);
}
__host__ __device__ inline float dec_bf16(uint16_t h) { return u2f(((uint32_t)h) << 16); }

// IEEE binary16 from float32, round to nearest even (software, exact).
__host__ __device__ inline uint16_t enc_fp16(float x) {
    uint32_t u = f2u(x);
    uint32_t sign = (u >> 16) & 0x8000u;
    uint32_t a = u & 0x7fffffffu;
    if (a > 0x7f800000u) return (uint16_t)(sign | 0x7e00u);          // NaN
    if (a >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);         // >= 65520 rounds to inf
    int e = (int)(a >> 23) - 127;
    if (e < -14) {                                                   // half subnormal (or zero)
        // value = q * 2^-24, q = rint(|x| * 2^24)
        float s = u2f(a) * 16777216.0f;                              // exact scaling
        float q = rintf(s);
        return (uint16_t)(sign | (uint32_t)q);                       // q = 1024 -> min normal
    }
    uint32_t mant = a & 0x7fffffu;
    uint32_t code = ((uint32_t)(e + 15) << 10) | (mant >> 13);
    uint32_t rem = mant & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (code & 1u))) code += 1u;
    return (uint16_t)(sign | code);
}
__host__ __device__ inline float dec_fp16(uint16_t h) {
    uint32_t sign = ((uint32_t)h & 0x8000u) << 16;
    uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    if (e == 0) {
        float v = (float)m * 5.9604644775390625e-08f;                // m * 2^-24, exact
        return u2f(f2u(v) | sign);
    }
    if (e == 31) return u2f(sign | 0x7f800000u | (m << 13));
    return u2f(sign | ((e - 15 + 127) << 23) | (m << 13));
}

// 8-bit floats with E exponent bits, M mantissa bits and exponent bias B,
// round to nearest even.  KIND 0: IEEE-style (top exponent holds inf / NaN);
// KIND 1: "fn" (finite, only S.1..1.1..1 is NaN); KIND 2: "fnuz" (finite, the
// negative-zero pattern 0x80 is NaN, zero is unsigned).  Past the largest
// finite value the result is inf (KIND 0) or NaN (KIND 1, 2), as a
// non-saturating conversion gives.
template <int E, int M, int B, int KIND>
__host__ __device__ inline uint8_t enc_f8(float x) {
    constexpr uint32_t EMAX = (1u << E) - 1, MMASK = (1u << M) - 1;
    constexpr uint32_t MAXCODE = KIND == 0 ? (((EMAX - 1) << M) | MMASK) : (KIND == 1 ? ((EMAX << M) | (MMASK - 1)) : 0x7fu);
    const uint32_t u = f2u(x);
    uint32_t sign = (u >> 24) & 0x80u;
    const uint32_t a = u & 0x7fffffffu;
    if (a > 0x7f800000u)                                              // NaN
        return KIND == 2 ? 0x80u : (KIND == 1 ? (uint8_t)(sign | 0x7fu) : (uint8_t)(sign | (EMAX << M) | (1u << (M - 1))));
    const int e = (int)(a >> 23) - 127;
    uint32_t code;
    if (e < 1 - B) {                                                  // below the smallest normal: subnormal
        const float q = rintf(u2f(a) * u2f((uint32_t)(B - 1 + M + 127) << 23));   // |x| / 2^(1-B-M), exact
        code = (uint32_t)q;                                           // q = 2^M is the smallest normal
    } else if (e + B > (int)EMAX + 1) {
        code = MAXCODE + 1;                                           // far past the range
    } else {
        const uint32_t mant = a & 0x7fffffu;
        code = ((uint32_t)(e + B) << M) | (mant >> (23 - M));
        const uint32_t rem = mant & ((1u << (23 - M)) - 1), half = 1u << (22 - M);
        if (rem > half || (rem == half && (code & 1u))) code += 1u;
    }
    if (code > MAXCODE) {
        if (KIND == 0) return (uint8_t)(sign | (EMAX << M));
        return KIND == 1 ? (uint8_t)(sign | 0x7fu) : 0x80u;
    }
    if (KIND == 2 && code == 0) sign = 0;
    return (uint8_t)(sign | code);
}

template <int E, int M, int B, int KIND>
__host__ __device__ inline float dec_f8(uint8_t c) {
    constexpr uint32_t EMAX = (1u << E) - 1, MMASK = (1u << M) - 1;
    const uint32_t sign = ((uint32_t)c & 0x80u) << 24;
    const uint32_t e = (c >> M) & EMAX, m = c & MMASK;
    if (KIND == 2 && c == 0x80u) return u2f(0x7fc00000u);
    if (KIND == 1 && e == EMAX && m == MMASK) return u2f(sign | 0x7fc00000u);
    if (KIND == 0 && e == EMAX) return u2f(sign | (m ? 0x7fc00000u : 0x7f800000u));
    const float v = e == 0 ? (float)m * u2f((uint32_t)(127 + 1 - B - M) << 23)          // m 2^(1-B-M)
                           : u2f(((e + 127 - B) << 23) | (m << (23 - M)));
    return u2f(f2u(v) | sign);
}

// OCP E4M3 (bias 7, max 448): the type of the scaled recorder.
__host__ __device__ inline uint8_t enc_e4m3(float x) { return enc_f8<4, 3, 7, 1>(x); }
__host__ __device__ inline float dec_e4m3(uint8_t c) { return dec_f8<4, 3, 7, 1>(c); }

// Power-of-two scale exponent: smallest e with 448 * 2^e >= m, clamped to [-126, 127].
__host__ __device__ inline int fp8_scale_exp(float m) {
    if (!(m > 0.0f)) return 0;
    uint32_t u = f2u(m);
    int E;
    uint32_t mant;
    if ((u >> 23) == 0) {                                            // float32 subnormal
        // m = mant * 2^-149; normalise
        uint32_t x = u & 0x7fffffu;
        int sh = 0;
        while (!(x & 0x800000u)) { x <<= 1; ++sh; }
        E = -126 - sh;                                               // m = 1.f * 2^E
        mant = x & 0x7fffffu;
    } else {
        E = (int)(u >> 23) - 127;
        mant = u & 0x7fffffu;
    }
    // m = 1.f * 2^E with 1.f in [1, 2), and 448 = 1.75 * 2^8, so
    //   448 * 2^e >= m  <=>  2^(e - E + 8) >= 1.f / 1.75, a ratio in [4/7, 8/7).
    // The smallest such e is E - 8 when 1.f <= 1.75 (mantissa <= 0x600000), else E - 7.
    int e = (mant > 0x600000u) ? E - 7 : E - 8;
    if (e < -126) e = -126;
    if (e > 127) e = 127;
    return e;
}

__host__ __device__ inline float pow2f(int e) {   // 2^e for e in [-126, 127]
    return u2f((uint32_t)(e + 127) << 23);
}

inline __host__ __device__ int storage_bytes(int dtype) {
    return dtype == 0 ? 4 : (dtype <= 2 ? 2 : 1);
}

// Storage types 4..9: the unscaled 8-bit types of the paper's comparison.
__device__ inline uint8_t enc_unscaled(int dtype, float v) {
    switch (dtype) {
        case 4: return enc_f8<4, 3, 11, 2>(v);   // e4m3b11fnuz
        case 5: return enc_f8<5, 2, 16, 2>(v);   // e5m2fnuz
        case 6: return enc_f8<4, 3, 8, 2>(v);    // e4m3fnuz
        case 7: return enc_f8<4, 3, 7, 0>(v);    // e4m3 (IEEE-style)
        case 8: return enc_f8<3, 4, 3, 0>(v);    // e3m4 (IEEE-style)
        default: return enc_f8<4, 3, 7, 1>(v);   // e4m3fn
    }
}
__device__ inline float dec_unscaled(int dtype, uint8_t c) {
    switch (dtype) {
        case 4: return dec_f8<4, 3, 11, 2>(c);
        case 5: return dec_f8<5, 2, 16, 2>(c);
        case 6: return dec_f8<4, 3, 8, 2>(c);
        case 7: return dec_f8<4, 3, 7, 0>(c);
        case 8: return dec_f8<3, 4, 3, 0>(c);
        default: return dec_f8<4, 3, 7, 1>(c);
    }
}

// ----------------------------------------------------------------------------
// Interface shell geometry: 12 blocks per kept step, in this order
//   0,1  x-low  (Hy, Hz) at i = P-1      [k][j]
//   2,3  y-low  (Hz, Hx) at j = P-1      [k][i]
//   4,5  z-low  (Hx, Hy) at k = P-1      [j][i]
//   6,7  x-high (Ey, Ez) at i = nx-P     [k][j]
//   8,9  y-high (Ez, Ex) at j = ny-P     [k][i]
//   10,11 z-high (Ex, Ey) at k = nz-P    [j][i]
// each over the interior extent of the other two axes.
// ----------------------------------------------------------------------------
__host__ __device__ inline long long block_offset(const Grid& g, int b) {
    // blocks 2f, 2f+1 of face f (x-, y-, z- low faces, then x+, y+, z+ high faces),
    // each as large as that face's plane; written without a local table so that a
    // run-time block index stays in registers
    const long long ax = (long long)g.my * g.mz, ay = (long long)g.mx * g.mz, az = (long long)g.mx * g.my;
    const int f = b >> 1, a = f % 3;
    const long long face = (f >= 3 ? 2 * (ax + ay + az) : 0) + (a >= 1 ? 2 * ax : 0) + (a >= 2 ? 2 * ay : 0);
    const long long area = a == 0 ? ax : (a == 1 ? ay : az);
    return face + (b & 1) * area;
}

__host__ __device__ inline long long block_len(const Grid& g, int b) {
    int f = (b >> 1) % 3;
    return f == 0 ? (long long)g.my * g.mz : (f == 1 ? (long long)g.mx * g.mz : (long long)g.mx * g.my);
}

// Face cell t of the interface shell on the low (high = false) or high faces, with
// t < my mz + mx mz + mx my (x face first, then y, then z): the cell (x, y, z), its
// two tangential components (c0, c1), the first of its two blocks (blk) and its
// position u within the block (block layouts as above).
struct FaceCell {
    int x, y, z, c0, c1, blk, u;
};
__device__ inline FaceCell face_cell(const Grid& g, int t, bool high) {
    const int P = g.P;
    const int ax = g.my * g.mz, ay = g.mx * g.mz;
    const int b0 = high ? 6 : 0;
    FaceCell f;
    if (t < ax) {
        f.u = t; f.blk = b0; f.y = P + f.u % g.my; f.z = P + f.u / g.my; f.x = high ? g.nx - P : P - 1;
        f.c0 = 1; f.c1 = 2;
    } else if (t < ax + ay) {
        f.u = t - ax; f.blk = b0 + 2; f.x = P + f.u % g.mx; f.z = P + f.u / g.mx; f.y = high ? g.ny - P : P - 1;
        f.c0 = 2; f.c1 = 0;
    } else {
        f.u = t - ax - ay; f.blk = b0 + 4; f.x = P + f.u % g.mx; f.y = P + f.u / g.mx; f.z = high ? g.nz - P : P - 1;
        f.c0 = 0; f.c1 = 1;
    }
    return f;
}

// Per-step parameters of the interpolating reinjection: v = sum_t w[t] * slice(j[t]) over
// the terms with j[t] >= 0 (j < 0: no term, or the exact zero anchor before the first
// step); two terms for linear interpolation, four for the cubic option.
struct Interp {
    int j[4];
    float w[4];
};

// The interface shell of one reverse step, written from the store into primal field
// buffers: E at the high faces (interpolation qE) into FE when do_e, H at the low
// faces (interpolation qH) into FH when do_h; with slice set, both into FE laid out as
// one kept step of the store (the intermediate step of a two-step reversal).
struct ShellJob {
    float* FE;
    float* FH;
    const void* store;
    Interp qE, qH;
    int do_e, do_h;
    int slice;
    int xrow;   // one-step reversal: x-face cells at position y - P of row 0 of their plane
};

// Compile-time storage type versions (the sweeps are instantiated per type so
// that no conversion code other than the one in use enters a kernel).
template <int DT>
__device__ inline float load_code_t(const void* store, long long byte_slice, long long off, float scale) {
    const char* base = (const char*)store + byte_slice;
    if constexpr (DT == 0) return ((const float*)base)[off];
    else if constexpr (DT == 1) return dec_fp16(((const uint16_t*)base)[off]);
    else if constexpr (DT == 2) return dec_bf16(((const uint16_t*)base)[off]);
    else if constexpr (DT == 3) return dec_e4m3(((const uint8_t*)base)[off]) * scale;
    else if constexpr (DT == 4) return dec_f8<4, 3, 11, 2>(((const uint8_t*)base)[off]);
    else if constexpr (DT == 5) return dec_f8<5, 2, 16, 2>(((const uint8_t*)base)[off]);
    else if constexpr (DT == 6) return dec_f8<4, 3, 8, 2>(((const uint8_t*)base)[off]);
    else if constexpr (DT == 7) return dec_f8<4, 3, 7, 0>(((const uint8_t*)base)[off]);
    else if constexpr (DT == 8) return dec_f8<3, 4, 3, 0>(((const uint8_t*)base)[off]);
    else return dec_f8<4, 3, 7, 1>(((const uint8_t*)base)[off]);
}

// One recorded value at element `elem` of a kept step (block offset + position):
// `dst` is the kept step's slice of the store, or for the scaled FP8 type the FP32
// staging buffer (quantised per block afterwards).
template <int DT>
__device__ inline void store_code(void* __restrict__ dst, long long elem, float v) {
    if constexpr (DT == 0 || DT == 3) {
        ((float*)dst)[elem] = v;
    } else if constexpr (DT == 1 || DT == 2) {
        ((uint16_t*)dst)[elem] = DT == 1 ? enc_fp16(v) : enc_bf16(v);
    } else {
        uint8_t q;
        if constexpr (DT == 4) q = enc_f8<4, 3, 11, 2>(v);
        else if constexpr (DT == 5) q = enc_f8<5, 2, 16, 2>(v);
        else if constexpr (DT == 6) q = enc_f8<4, 3, 8, 2>(v);
        else if constexpr (DT == 7) q = enc_f8<4, 3, 7, 0>(v);
        else if constexpr (DT == 8) q = enc_f8<3, 4, 3, 0>(v);
        else q = enc_f8<4, 3, 7, 1>(v);
        ((uint8_t*)dst)[elem] = q;
    }
}

template <int DT>
__device__ inline float shell_value_t(const Grid& g, const void* store, const Interp& q, int b, long long off) {
    const long long o = block_offset(g, b) + off;
    const float* scales = (const float*)((const char*)store + g.scale_off);
    float v = 0.0f;
    #pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (q.j[t] >= 0) {
            const float s = DT == 3 ? scales[q.j[t] * 12 + b] : 1.0f;
            v += q.w[t] * load_code_t<DT>(store, q.j[t] * g.slice_stride, o, s);
        }
    }
    return v;
}

// Calls f.template operator()<DT>() with the storage type as a compile-time constant.
template <class F>
inline void with_dtype(int dtype, F&& f) {
    switch (dtype) {
        case 0: f.template operator()<0>(); break;
        case 1: f.template operator()<1>(); break;
        case 2: f.template operator()<2>(); break;
        case 3: f.template operator()<3>(); break;
        case 4: f.template operator()<4>(); break;
        case 5: f.template operator()<5>(); break;
        case 6: f.template operator()<6>(); break;
        case 7: f.template operator()<7>(); break;
        case 8: f.template operator()<8>(); break;
        default: f.template operator()<9>(); break;
    }
}

__device__ inline bool in_box(int i, int j, int k, const int lo[3], const int hi[3]) {
    return i >= lo[0] && i < hi[0] && j >= lo[1] && j < hi[1] && k >= lo[2] && k < hi[2];
}

// Neighbour at +1 along an axis (zero outside, or wrapped)
__device__ inline float nb_plus(const float* f, long long idx, int i, int n, long long stride, int periodic) {
    if (i + 1 < n) return f[idx + stride];
    return periodic ? f[idx - (long long)(n - 1) * stride] : 0.0f;
}
__device__ inline float nb_minus(const float* f, long long idx, int i, int n, long long stride, int periodic) {
    if (i > 0) return f[idx - stride];
    return periodic ? f[idx + (long long)(n - 1) * stride] : 0.0f;
}

// One step's loss term at one detector cell from E^{n+1} and H^{n+1/2} at that index:
// |E|^2 (loss 0) or (E x H) along x, y, z (loss 1, 2, 3).  Written without run-time
// array indices so that e and h stay in registers.
__device__ inline double loss_term(int loss, const float e[3], const float h[3]) {
    switch (loss) {
        case 1: return (double)e[1] * h[2] - (double)e[2] * h[1];
        case 2: return (double)e[2] * h[0] - (double)e[0] * h[2];
        case 3: return (double)e[0] * h[1] - (double)e[1] * h[0];
        default: return (double)e[0] * e[0] + (double)e[1] * e[1] + (double)e[2] * e[2];
    }
}

// Its derivatives (dL/dE^{n+1}, dL/dH^{n+1/2}) at that cell.
__device__ inline void loss_seeds(int loss, const float e[3], const float h[3], float gE[3], float gH[3]) {
    gE[0] = gE[1] = gE[2] = gH[0] = gH[1] = gH[2] = 0.0f;
    switch (loss) {
        case 1: gE[1] = h[2]; gE[2] = -h[1]; gH[2] = e[1]; gH[1] = -e[2]; break;
        case 2: gE[2] = h[0]; gE[0] = -h[2]; gH[0] = e[2]; gH[2] = -e[0]; break;
        case 3: gE[0] = h[1]; gE[1] = -h[0]; gH[1] = e[0]; gH[0] = -e[1]; break;
        default: gE[0] = 2.0f * e[0]; gE[1] = 2.0f * e[1]; gE[2] = 2.0f * e[2]; break;
    }
}

// The owner of an interior cell on the design or detector box: this step's loss
// derivatives (2 E^{n+1} for |E|^2; H- and E-terms for a flux) are added to Ebar and
// Hbar in place (the adjoint sweep reads them seeded), and the gradient
// epsbar -= (dt/eps^2) Ebar . (U - J) accumulates in FP64.  Eb0 is the adjoint field
// buffer (Ebar, then Hbar at component stride g.N).
__device__ inline void grad_and_seed(const Grid& g, float* __restrict__ Eb0, double* __restrict__ grad,
                                              int x, int y, int z, int idx, const float e1[3], const float h[3],
                                              float ep, const float u[3]) {
    const bool det = in_box(x, y, z, g.det_lo, g.det_hi), des = in_box(x, y, z, g.des_lo, g.des_hi);
    if (!det && !des) return;
    const long long N = g.N;
    float eb[3] = {Eb0[idx], Eb0[N + idx], Eb0[2 * N + idx]};
    if (det) {
        float gE[3], gH[3];
        loss_seeds(g.loss, e1, h, gE, gH);
        eb[0] += gE[0];
        eb[1] += gE[1];
        eb[2] += gE[2];
        Eb0[idx] = eb[0];
        Eb0[N + idx] = eb[1];
        Eb0[2 * N + idx] = eb[2];
        if (g.loss != 0) {
            float* Hb0 = Eb0 + 3 * N;
            Hb0[idx] += gH[0];
            Hb0[N + idx] += gH[1];
            Hb0[2 * N + idx] += gH[2];
        }
    }
    if (des) {
        const int dx = g.des_hi[0] - g.des_lo[0], dy = g.des_hi[1] - g.des_lo[1];
        const int di = (x - g.des_lo[0]) + dx * ((y - g.des_lo[1]) + dy * (z - g.des_lo[2]));
        const double ee = (double)ep;
        const double s = (double)eb[0] * u[0] + (double)eb[1] * u[1] + (double)eb[2] * u[2];
        grad[di] -= (double)g.dt / (ee * ee) * s;
    }
}

// dt / eps of the E update; the forward step, its reversal and its adjoint all use
// this one expression, so that they agree bit for bit.
__device__ inline float dt_over_eps(float dt, float ep) { return __fdividef(dt, ep); }

__device__ inline int slab_coord(int i, int n, int P) {   // -1 outside the slab
    if (i < P) return i;
    if (i >= n - P) return i - (n - 2 * P);
    return -1;
}

// ----------------------------------------------------------------------------
// Launches.  With per-kernel timing on, each launch carries a start and stop
// event on its own dispatch (hipExtLaunchKernelGGL), so the recorded interval
// is the kernel's execution and no extra packet enters the stream.
// ----------------------------------------------------------------------------
enum KernelKind {
    K_FILL = 0, K_FWD_STEP, K_REC_QUANT, K_LOSS_FINAL, K_INJECT, K_PRIM_REV, K_ADJ_STEP, K_SCALE_GRAD,
    K_CODEC, K_PUT, K_RECORD, K_FWD_STEP2, K_PRIM_REV2, K_REV_PENDING, K_NUM_KINDS
};

// Defined in api.hip: hands out an event pair when timing is enabled.
bool timing_acquire(int kind, hipEvent_t* start, hipEvent_t* stop);

template <typename Kernel, typename... Args>
inline void launch_kernel(int kind, Kernel kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
    hipEvent_t a, b;
    if (timing_acquire(kind, &a, &b))
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// Launch wrappers (defined with the kernels)
constexpr int PUT_CHUNK = 896;        // 32-bit words carried by one k_put launch (3.5 KB of arguments)
void launch_put(void* dst, const void* host, long long n, hipStream_t s);
void launch_fill(float* p, long long n, float v, hipStream_t s);
void launch_fill_f64(double* p, long long n, double v, hipStream_t s);
struct Tiling;
// Interface values of kept steps recorded from one field buffer F (E then H): E on the
// high faces into the store's kept step dst_e, H on the low faces into dst_h (a null
// destination skips that side).  Stored in the storage type directly (not for the
// scaled FP8 type, which goes through the staging buffer and its own launches).
struct RecJob {
    const float* F;
    void* dst_e;
    void* dst_h;
};
// job (may be NULL): kept-step values recorded by trailing workgroups of the same launch
void launch_fwd_step(const Grid& g, const Tiling& t, const float* F0, float* F1, float* psi, int hcopy,
                     const float* eps, float wave, float mwave, double* partials, const RecJob* job, hipStream_t s);
// a RecJob as a launch of its own
void launch_record_job(const Grid& g, const RecJob& job, hipStream_t s);
// two forward steps n, n+1 in one sweep (PML copies: H side hcopy, E side ecopy in;
// the other copies out); p0, p1: the two steps' detector partials; mid: NULL or the
// buffer that receives the intermediate step's recorder values
void launch_fwd2_step(const Grid& g, const Tiling& t, const float* F0, float* F1, float* psi, int hcopy, int ecopy,
                      const float* eps, float w0, float w1, double* p0, double* p1, float* mid, hipStream_t s);
// recorder of kept step `slice` of forward step n: E^n on the high faces from E (a field
// buffer, or when e_mid a buffer laid out as one kept step), H^{n+1/2} on the low faces
// from H (likewise with h_mid)
void launch_record(const Grid& g, const float* E, bool e_mid, const float* H, bool h_mid, void* store,
                   float* staging, int slice, hipStream_t s);
// scaled FP8 recorder: the staging values of one kept step, then the chunk maxima
long long rec_quant_scratch_floats(const Grid& g);
void launch_rec_quant(const Grid& g, const float* staging, void* store, int slice, hipStream_t s);
void launch_loss_final(const double* partials, int steps, int per_step, double* loss, double* series,
                       hipStream_t s);
void launch_inject_shell(const Grid& g, const ShellJob& job, hipStream_t s);
// two reverse steps n, n-1 of the primal interior in one sweep (F0 -> F1), with step n's
// gradient and loss seed (adjoint E of step n in Eb0) and, for step n-1, the values its
// seed and gradient need kept in stash; mid: step n's interface shell (one kept step)
void launch_rev2(const Grid& g, const Tiling& t, const float* F0, float* F1, const float* eps, float* Eb0,
                 float wave_n, float wave_n1, double* grad, float* stash, const float* mid, hipStream_t s);
// step n-1's loss seed into the adjoint fields A (E then H) and its gradient term, from stash
void launch_rev_pending(const Grid& g, float* A, double* grad, const float* stash, hipStream_t s);
// xrow: the x-face shell cells sit at position y - P of row 0 of their plane (ShellJob.xrow)
void launch_prim_rev(const Grid& g, const Tiling& t, const int box_o[3], const int box_n[3], int tile_x0, int xrow,
                     const float* F0, float* F1, const float* eps, float* Eb0, float wave, float mwave,
                     double* grad, hipStream_t s);
// job (may be NULL): a shell written by trailing workgroups of the same launch
void launch_adj_step(const Grid& g, const Tiling& t, const float* A0, float* A1, const float* eps, float* psi,
                     int pcopy, const ShellJob* job, hipStream_t s);
void launch_scale_grad(double* grad, long long n, const double* scale, hipStream_t s);
void launch_codec_roundtrip(int dtype, const float* values, long long n_blocks, long long block_len,
                            void* codes, float* scales, float* decoded, hipStream_t s);

}  // namespace fdtd
