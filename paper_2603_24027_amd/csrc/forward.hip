// Forward Yee step with convolutional PML, interface recorder and detector loss (gfx950).
//
// One step n is two sweeps over the grid (one thread per cell, x fastest,
// 64 x 4 threads per block):
//   fwd_h  H^{n+1/2} = H^{n-1/2} - dt curl E^n         (forward differences)
//          and, on kept steps, the interface shell: E^n on the high faces and
//          H^{n+1/2} on the low faces (Section 2: the interface slices are
//          recorded during the forward simulation)
//   fwd_e  E^{n+1} = E^n + (dt / eps)(curl H^{n+1/2} - J^n)  (backward differences)
//          and the per-block FP64 partial of sum_D |E^{n+1}|^2
// The PML recursions psi <- b psi + a g run only inside the slabs.
#include "common.h"

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

__global__ __launch_bounds__(BX * BY) void k_fwd_h(Grid g, const float* __restrict__ E, float* __restrict__ H,
                                                   float* __restrict__ psi, void* __restrict__ store,
                                                   float* __restrict__ staging, int slice) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const long long N = g.N;
    const long long sy = g.nx, sz = (long long)g.nx * g.ny;
    const long long idx = i + sy * j + sz * k;
    const float* Ex = E;
    const float* Ey = E + N;
    const float* Ez = E + 2 * N;
    const float ex = Ex[idx], ey = Ey[idx], ez = Ez[idx];
    const float ey_xp = nb_plus(Ey, idx, i, g.nx, 1, g.periodic);
    const float ez_xp = nb_plus(Ez, idx, i, g.nx, 1, g.periodic);
    const float ex_yp = nb_plus(Ex, idx, j, g.ny, sy, g.periodic);
    const float ez_yp = nb_plus(Ez, idx, j, g.ny, sy, g.periodic);
    const float ex_zp = nb_plus(Ex, idx, k, g.nz, sz, g.periodic);
    const float ey_zp = nb_plus(Ey, idx, k, g.nz, sz, g.periodic);

    float t0 = ez_yp - ez;   // (Hx, y, +, Ez)
    float t1 = ey_zp - ey;   // (Hx, z, -, Ey)
    float t2 = ex_zp - ex;   // (Hy, z, +, Ex)
    float t3 = ez_xp - ez;   // (Hy, x, -, Ez)
    float t4 = ey_xp - ey;   // (Hz, x, +, Ey)
    float t5 = ex_yp - ex;   // (Hz, y, -, Ex)

    const int P = g.P;
    if (P > 0) {
        const float* bH = g.coef + 6 * P;
        const float* aH = g.coef + 8 * P;
        const float* kH = g.coef + 10 * P;
        int s = slab_coord(i, g.nx, P);
        if (s >= 0) {
            long long o = g.psi_off[0] + s + 2LL * P * (j + (long long)g.ny * k);
            float b = bH[s], a = aH[s], kv = kH[s];
            float p3 = b * psi[o] + a * t3;
            float p4 = b * psi[o + g.slab[0]] + a * t4;
            psi[o] = p3;
            psi[o + g.slab[0]] = p4;
            t3 = kv * t3 + p3;
            t4 = kv * t4 + p4;
        }
        s = slab_coord(j, g.ny, P);
        if (s >= 0) {
            long long o = g.psi_off[1] + i + (long long)g.nx * (s + 2LL * P * k);
            float b = bH[s], a = aH[s], kv = kH[s];
            float p0 = b * psi[o] + a * t0;
            float p5 = b * psi[o + g.slab[1]] + a * t5;
            psi[o] = p0;
            psi[o + g.slab[1]] = p5;
            t0 = kv * t0 + p0;
            t5 = kv * t5 + p5;
        }
        s = slab_coord(k, g.nz, P);
        if (s >= 0) {
            long long o = g.psi_off[2] + i + (long long)g.nx * (j + (long long)g.ny * s);
            float b = bH[s], a = aH[s], kv = kH[s];
            float p1 = b * psi[o] + a * t1;
            float p2 = b * psi[o + g.slab[2]] + a * t2;
            psi[o] = p1;
            psi[o + g.slab[2]] = p2;
            t1 = kv * t1 + p1;
            t2 = kv * t2 + p2;
        }
    }
    float* Hx = H;
    float* Hy = H + N;
    float* Hz = H + 2 * N;
    const float dt = g.dt;
    const float hx = Hx[idx] - dt * (t0 - t1);
    const float hy = Hy[idx] - dt * (t2 - t3);
    const float hz = Hz[idx] - dt * (t4 - t5);
    Hx[idx] = hx;
    Hy[idx] = hy;
    Hz[idx] = hz;

    if (slice >= 0 && P > 0) {
        // interface shell of a kept step: H^{n+1/2} on the low faces, E^n on the high faces
        const bool jI = j >= P && j < g.ny - P, kI = k >= P && k < g.nz - P, iI = i >= P && i < g.nx - P;
        const long long bs = (long long)slice * g.slice_stride;
        const int dt_ = g.dtype;
        float* st = staging;
        auto put = [&](int b, long long off, float v) {
            long long o = block_offset(g, b) + off;
            if (dt_ == 3) st[o] = v; else store_code(store, bs, o, dt_, v);
        };
        if (i == P - 1 && jI && kI) {
            long long off = (long long)(k - P) * g.my + (j - P);
            put(0, off, hy); put(1, off, hz);
        }
        if (j == P - 1 && iI && kI) {
            long long off = (long long)(k - P) * g.mx + (i - P);
            put(2, off, hz); put(3, off, hx);
        }
        if (k == P - 1 && iI && jI) {
            long long off = (long long)(j - P) * g.mx + (i - P);
            put(4, off, hx); put(5, off, hy);
        }
        if (i == g.nx - P && jI && kI) {
            long long off = (long long)(k - P) * g.my + (j - P);
            put(6, off, ey); put(7, off, ez);
        }
        if (j == g.ny - P && iI && kI) {
            long long off = (long long)(k - P) * g.mx + (i - P);
            put(8, off, ez); put(9, off, ex);
        }
        if (k == g.nz - P && iI && jI) {
            long long off = (long long)(j - P) * g.mx + (i - P);
            put(10, off, ex); put(11, off, ey);
        }
    }
}

__global__ __launch_bounds__(BX * BY) void k_fwd_e(Grid g, float* __restrict__ E, const float* __restrict__ H,
                                                   const float* __restrict__ eps, float* __restrict__ psi,
                                                   float wave, double* __restrict__ partials) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    const bool live = i < g.nx && j < g.ny;
    double e2 = 0.0;
    if (live) {
        const long long N = g.N;
        const long long sy = g.nx, sz = (long long)g.nx * g.ny;
        const long long idx = i + sy * j + sz * k;
        const float* Hx = H;
        const float* Hy = H + N;
        const float* Hz = H + 2 * N;
        const float hx = Hx[idx], hy = Hy[idx], hz = Hz[idx];
        const float hz_xm = nb_minus(Hz, idx, i, g.nx, 1, g.periodic);
        const float hy_xm = nb_minus(Hy, idx, i, g.nx, 1, g.periodic);
        const float hz_ym = nb_minus(Hz, idx, j, g.ny, sy, g.periodic);
        const float hx_ym = nb_minus(Hx, idx, j, g.ny, sy, g.periodic);
        const float hy_zm = nb_minus(Hy, idx, k, g.nz, sz, g.periodic);
        const float hx_zm = nb_minus(Hx, idx, k, g.nz, sz, g.periodic);

        float t0 = hz - hz_ym;   // (Ex, y, +, Hz)
        float t1 = hy - hy_zm;   // (Ex, z, -, Hy)
        float t2 = hx - hx_zm;   // (Ey, z, +, Hx)
        float t3 = hz - hz_xm;   // (Ey, x, -, Hz)
        float t4 = hy - hy_xm;   // (Ez, x, +, Hy)
        float t5 = hx - hx_ym;   // (Ez, y, -, Hx)

        const int P = g.P;
        if (P > 0) {
            const float* bE = g.coef;
            const float* aE = g.coef + 2 * P;
            const float* kE = g.coef + 4 * P;
            int s = slab_coord(i, g.nx, P);
            if (s >= 0) {
                long long o = g.psi_off[0] + 2 * g.slab[0] + s + 2LL * P * (j + (long long)g.ny * k);
                float b = bE[s], a = aE[s], kv = kE[s];
                float p3 = b * psi[o] + a * t3;
                float p4 = b * psi[o + g.slab[0]] + a * t4;
                psi[o] = p3;
                psi[o + g.slab[0]] = p4;
                t3 = kv * t3 + p3;
                t4 = kv * t4 + p4;
            }
            s = slab_coord(j, g.ny, P);
            if (s >= 0) {
                long long o = g.psi_off[1] + 2 * g.slab[1] + i + (long long)g.nx * (s + 2LL * P * k);
                float b = bE[s], a = aE[s], kv = kE[s];
                float p0 = b * psi[o] + a * t0;
                float p5 = b * psi[o + g.slab[1]] + a * t5;
                psi[o] = p0;
                psi[o + g.slab[1]] = p5;
                t0 = kv * t0 + p0;
                t5 = kv * t5 + p5;
            }
            s = slab_coord(k, g.nz, P);
            if (s >= 0) {
                long long o = g.psi_off[2] + 2 * g.slab[2] + i + (long long)g.nx * (j + (long long)g.ny * s);
                float b = bE[s], a = aE[s], kv = kE[s];
                float p1 = b * psi[o] + a * t1;
                float p2 = b * psi[o + g.slab[2]] + a * t2;
                psi[o] = p1;
                psi[o + g.slab[2]] = p2;
                t1 = kv * t1 + p1;
                t2 = kv * t2 + p2;
            }
        }
        float ux = t0 - t1, uy = t2 - t3, uz = t4 - t5;
        if (in_box(i, j, k, g.src_lo, g.src_hi)) {
            const int sxn = g.src_hi[0] - g.src_lo[0], syn = g.src_hi[1] - g.src_lo[1];
            const float jv = wave * g.src_profile[(i - g.src_lo[0]) + (long long)sxn *
                                                  ((j - g.src_lo[1]) + (long long)syn * (k - g.src_lo[2]))];
            if (g.src_comp == 0) ux -= jv; else if (g.src_comp == 1) uy -= jv; else uz -= jv;
        }
        const float c = g.dt / eps[idx];
        float* Ex = E;
        float* Ey = E + N;
        float* Ez = E + 2 * N;
        const float ex = Ex[idx] + c * ux;
        const float ey = Ey[idx] + c * uy;
        const float ez = Ez[idx] + c * uz;
        Ex[idx] = ex;
        Ey[idx] = ey;
        Ez[idx] = ez;
        if (in_box(i, j, k, g.det_lo, g.det_hi))
            e2 = (double)ex * ex + (double)ey * ey + (double)ez * ez;
    }
    // detector partial of this block (blocks intersecting the detector only; uniform test)
    const int bx = blockIdx.x - g.dbx0, by = blockIdx.y - g.dby0, bz = blockIdx.z - g.dbz0;
    if (bx < 0 || by < 0 || bz < 0 || bx >= g.dnbx || by >= g.dnby || bz >= g.dnbz) return;
    __shared__ double red[BY];
    for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off, 64);
    const int lane = threadIdx.x;   // BX == 64: one wavefront per threadIdx.y
    if (lane == 0) red[threadIdx.y] = e2;
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double sum = 0.0;
        for (int w = 0; w < BY; ++w) sum += red[w];
        partials[(long long)bx + (long long)g.dnbx * (by + (long long)g.dnby * bz)] = sum;
    }
}

// FP8 recorder: one block per (face, component) block of a kept step.  absmax
// (exact: max does not round), power-of-two scale, E4M3 codes.
__global__ __launch_bounds__(256) void k_rec_quant(Grid g, const float* __restrict__ staging,
                                                   void* __restrict__ store, int slice) {
    const int b = blockIdx.x;
    const long long off = block_offset(g, b), len = block_len(g, b);
    const float* x = staging + off;
    float m = 0.0f;
    for (long long t = threadIdx.x; t < len; t += 256) m = fmaxf(m, fabsf(x[t]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    __shared__ float red[4];
    __shared__ float sc;
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float mm = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        sc = pow2f(fp8_scale_exp(mm));
        ((float*)((char*)store + g.scale_off))[slice * 12 + b] = sc;
    }
    __syncthreads();
    const float inv = 1.0f / sc;   // exact: sc is a power of two in the normal range
    uint8_t* q = (uint8_t*)store + (long long)slice * g.slice_stride + off;
    for (long long t = threadIdx.x; t < len; t += 256) q[t] = enc_e4m3(x[t] * inv);
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

static dim3 grid_dims(const Grid& g) {
    return dim3((unsigned)((g.nx + BX - 1) / BX), (unsigned)((g.ny + BY - 1) / BY), (unsigned)g.nz);
}

void launch_fwd_h(const Grid& g, const float* E, float* H, float* psi, void* store, float* staging,
                  int slice, hipStream_t s) {
    launch_kernel(K_FWD_H, k_fwd_h, grid_dims(g), dim3(BX, BY), s, g, E, H, psi, store, staging, slice);
}

void launch_fwd_e(const Grid& g, float* E, const float* H, const float* eps, float* psi, float wave,
                  double* partials, hipStream_t s) {
    launch_kernel(K_FWD_E, k_fwd_e, grid_dims(g), dim3(BX, BY), s, g, E, H, eps, psi, wave, partials);
}

void launch_rec_quant(const Grid& g, const float* staging, void* store, int slice, hipStream_t s) {
    launch_kernel(K_REC_QUANT, k_rec_quant, dim3(12), dim3(256), s, g, staging, store, slice);
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
        } else {
            uint16_t c = enc_bf16(v);
            ((uint16_t*)codes)[b * len + t] = c;
            ob[t] = dec_bf16(c);
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
