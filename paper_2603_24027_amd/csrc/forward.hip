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
#include "march.h"

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

// H^{n+1/2} at one cell from the LDS planes of E^n at z (cur) and z + 1 (nxt).
// (ex, ey): extended-plane coordinates; (x, y, z): the cell's index inside the
// domain.  PML auxiliaries are read from psi_in and, for the owning block,
// written to psi_out (NULL for a recomputed halo cell).
template <int TY>
__device__ inline void h_cell(const Grid& g, const float (*cur)[TY + 2][EXT], const float (*nxt)[TY + 2][EXT],
                              int ex, int ey, int x, int y, int z, const float* __restrict__ H0,
                              const float* __restrict__ psi_in, float* __restrict__ psi_out,
                              float& hx, float& hy, float& hz) {
    const float exc = cur[0][ey][ex], eyc = cur[1][ey][ex], ezc = cur[2][ey][ex];
    float t0 = cur[2][ey + 1][ex] - ezc;   // (Hx, y, +, Ez)
    float t1 = nxt[1][ey][ex] - eyc;       // (Hx, z, -, Ey)
    float t2 = nxt[0][ey][ex] - exc;       // (Hy, z, +, Ex)
    float t3 = cur[2][ey][ex + 1] - ezc;   // (Hy, x, -, Ez)
    float t4 = cur[1][ey][ex + 1] - eyc;   // (Hz, x, +, Ey)
    float t5 = cur[0][ey + 1][ex] - exc;   // (Hz, y, -, Ex)
    const int P = g.P;
    if (P > 0) {
        const float* bH = g.coef + 6 * P;
        const float* aH = g.coef + 8 * P;
        const float* kH = g.coef + 10 * P;
        int s = slab_coord(x, g.nx, P);
        if (s >= 0) {
            const int o = (int)g.psi_off[0] + s + 2 * P * (y + g.ny * z);
            const float b = bH[s], a = aH[s], kv = kH[s];
            const float p3 = b * psi_in[o] + a * t3;
            const float p4 = b * psi_in[o + (int)g.slab[0]] + a * t4;
            if (psi_out) { psi_out[o] = p3; psi_out[o + (int)g.slab[0]] = p4; }
            t3 = kv * t3 + p3;
            t4 = kv * t4 + p4;
        }
        s = slab_coord(y, g.ny, P);
        if (s >= 0) {
            const int o = (int)g.psi_off[1] + x + g.nx * (s + 2 * P * z);
            const float b = bH[s], a = aH[s], kv = kH[s];
            const float p0 = b * psi_in[o] + a * t0;
            const float p5 = b * psi_in[o + (int)g.slab[1]] + a * t5;
            if (psi_out) { psi_out[o] = p0; psi_out[o + (int)g.slab[1]] = p5; }
            t0 = kv * t0 + p0;
            t5 = kv * t5 + p5;
        }
        s = slab_coord(z, g.nz, P);
        if (s >= 0) {
            const int o = (int)g.psi_off[2] + x + g.nx * (y + g.ny * s);
            const float b = bH[s], a = aH[s], kv = kH[s];
            const float p1 = b * psi_in[o] + a * t1;
            const float p2 = b * psi_in[o + (int)g.slab[2]] + a * t2;
            if (psi_out) { psi_out[o] = p1; psi_out[o + (int)g.slab[2]] = p2; }
            t1 = kv * t1 + p1;
            t2 = kv * t2 + p2;
        }
    }
    const int N = (int)g.N;
    const int idx = x + g.nx * (y + g.ny * z);
    const float dt = g.dt;
    hx = H0[idx] - dt * (t0 - t1);
    hy = H0[N + idx] - dt * (t2 - t3);
    hz = H0[2 * N + idx] - dt * (t4 - t5);
}

// One full forward step n: (E^n, H^{n-1/2}) in E0/H0 -> (E^{n+1}, H^{n+1/2}) in E1/H1.
// H-side PML auxiliaries ping-pong (psiH0 -> psiH1); E-side ones are updated in place.
template <int TY>
__global__ __launch_bounds__(TX * TY) void k_fwd_step(Grid g, Tiling tl, const float* __restrict__ E0,
                                                      const float* __restrict__ H0, float* __restrict__ E1,
                                                      float* __restrict__ H1, const float* __restrict__ psiH0,
                                                      float* __restrict__ psiH1, float* __restrict__ psiE,
                                                      const float* __restrict__ eps, float wave,
                                                      double* __restrict__ partials, void* __restrict__ store,
                                                      float* __restrict__ staging, int slice) {
    __shared__ float sE[2][3][TY + 2][EXT];
    __shared__ float sH[3][TY + 1][TX + 1];
    __shared__ double red[TY];
    const int L = logical_tile(tl.count);
    const int tix = L % tl.ntx, tiy = (L / tl.ntx) % tl.nty, tiz = L / (tl.ntx * tl.nty);
    const int i0 = tix * TX, j0 = tiy * TY, k0 = tiz * tl.cz;
    const int k1 = min(k0 + tl.cz, g.nz);
    const int lane = threadIdx.x, row = threadIdx.y;
    const int tid = row * TX + lane;
    const int x = i0 + lane, y = j0 + row;
    const bool live = x < g.nx && y < g.ny;
    const int N = (int)g.N;
    const int P = g.P;

    // halo cell of the first half assigned to this thread: the row below the tile (y = j0-1)
    // for tid < TX, the column left of it (x = i0-1) for TX <= tid < TX + TY
    int hex = -1, hey = -1, hxg = -1, hyg = -1;
    if (tid < TX + TY) {
        if (tid < TX) { hex = tid + 1; hey = 0; } else { hex = 0; hey = tid - TX + 1; }
        const int xr = i0 - 1 + hex, yr = j0 - 1 + hey;
        if (xr < g.nx && yr < g.ny) {
            hxg = bound(xr, g.nx, g.periodic);
            hyg = bound(yr, g.ny, g.periodic);
        }
    }

    // prologue: H^{n+1/2} of this column at k0 - 1 (the owner below computes the same value)
    load_ext_plane<TY>(sE[0], E0, N, g, i0, j0, k0 - 1);
    load_ext_plane<TY>(sE[1], E0, N, g, i0, j0, k0);
    __syncthreads();
    float hx_prev = 0.0f, hy_prev = 0.0f;
    {
        const int zb = bound(k0 - 1, g.nz, g.periodic);
        if (live && zb >= 0) {
            float a, b, c;
            h_cell<TY>(g, sE[0], sE[1], lane + 1, row + 1, x, y, zb, H0, psiH0, nullptr, a, b, c);
            hx_prev = a;
            hy_prev = b;
        }
    }
    int cur = 1;
    double e2 = 0.0;
    const bool rec = slice >= 0 && P > 0;
    const long long bs = (long long)slice * g.slice_stride;
    for (int k = k0; k < k1; ++k) {
        const int nxt = 1 - cur;
        __syncthreads();                                   // sE[nxt] and sH are free
        load_ext_plane<TY>(sE[nxt], E0, N, g, i0, j0, k + 1);
        __syncthreads();
        float hx = 0.0f, hy = 0.0f, hz = 0.0f;
        const int idx = x + g.nx * (y + g.ny * k);
        // pass 0: this thread's own cell; pass 1: its halo cell (if any).  One code path for
        // both keeps a recomputed halo value bitwise equal to the owner's.
        #pragma unroll 1
        for (int pass = 0; pass < 2; ++pass) {
            const bool own = pass == 0;
            const bool active = own ? live : (hxg >= 0 && hyg >= 0);
            const int cex = own ? lane + 1 : hex, cey = own ? row + 1 : hey;
            const int cx = own ? x : hxg, cy = own ? y : hyg;
            if (!own && hex < 0) break;
            float a = 0.0f, b = 0.0f, c = 0.0f;
            if (active)
                h_cell<TY>(g, sE[cur], sE[nxt], cex, cey, cx, cy, k, H0, psiH0, own ? psiH1 : nullptr, a, b, c);
            sH[0][cey][cex] = a;
            sH[1][cey][cex] = b;
            sH[2][cey][cex] = c;
            if (own) { hx = a; hy = b; hz = c; }
        }
        if (live) {
            H1[idx] = hx;
            H1[N + idx] = hy;
            H1[2 * N + idx] = hz;
            if (rec) {
                // interface shell of a kept step: H^{n+1/2} on the low faces, E^n on the high faces
                const float exo = sE[cur][0][row + 1][lane + 1];
                const float eyo = sE[cur][1][row + 1][lane + 1];
                const float ezo = sE[cur][2][row + 1][lane + 1];
                const bool jI = y >= P && y < g.ny - P, kI = k >= P && k < g.nz - P, iI = x >= P && x < g.nx - P;
                auto put = [&](int b, int off, float v) {
                    const long long o = block_offset(g, b) + off;
                    if (g.dtype == 3) staging[o] = v; else store_code(store, bs, o, g.dtype, v);
                };
                if (x == P - 1 && jI && kI) { const int o = (k - P) * g.my + (y - P); put(0, o, hy); put(1, o, hz); }
                if (y == P - 1 && iI && kI) { const int o = (k - P) * g.mx + (x - P); put(2, o, hz); put(3, o, hx); }
                if (k == P - 1 && iI && jI) { const int o = (y - P) * g.mx + (x - P); put(4, o, hx); put(5, o, hy); }
                if (x == g.nx - P && jI && kI) { const int o = (k - P) * g.my + (y - P); put(6, o, eyo); put(7, o, ezo); }
                if (y == g.ny - P && iI && kI) { const int o = (k - P) * g.mx + (x - P); put(8, o, ezo); put(9, o, exo); }
                if (k == g.nz - P && iI && jI) { const int o = (y - P) * g.mx + (x - P); put(10, o, exo); put(11, o, eyo); }
            }
        }
        __syncthreads();
        if (live) {
            float t0 = hz - sH[2][row][lane + 1];       // (Ex, y, +, Hz)
            float t1 = hy - hy_prev;                    // (Ex, z, -, Hy)
            float t2 = hx - hx_prev;                    // (Ey, z, +, Hx)
            float t3 = hz - sH[2][row + 1][lane];       // (Ey, x, -, Hz)
            float t4 = hy - sH[1][row + 1][lane];       // (Ez, x, +, Hy)
            float t5 = hx - sH[0][row][lane + 1];       // (Ez, y, -, Hx)
            if (P > 0) {
                const float* bE = g.coef;
                const float* aE = g.coef + 2 * P;
                const float* kE = g.coef + 4 * P;
                int s = slab_coord(x, g.nx, P);
                if (s >= 0) {
                    const int o = (int)(g.psi_off[0] + 2 * g.slab[0]) + s + 2 * P * (y + g.ny * k);
                    const int sl = (int)g.slab[0];
                    const float b = bE[s], a = aE[s], kv = kE[s];
                    const float p3 = b * psiE[o] + a * t3;
                    const float p4 = b * psiE[o + sl] + a * t4;
                    psiE[o] = p3;
                    psiE[o + sl] = p4;
                    t3 = kv * t3 + p3;
                    t4 = kv * t4 + p4;
                }
                s = slab_coord(y, g.ny, P);
                if (s >= 0) {
                    const int o = (int)(g.psi_off[1] + 2 * g.slab[1]) + x + g.nx * (s + 2 * P * k);
                    const int sl = (int)g.slab[1];
                    const float b = bE[s], a = aE[s], kv = kE[s];
                    const float p0 = b * psiE[o] + a * t0;
                    const float p5 = b * psiE[o + sl] + a * t5;
                    psiE[o] = p0;
                    psiE[o + sl] = p5;
                    t0 = kv * t0 + p0;
                    t5 = kv * t5 + p5;
                }
                s = slab_coord(k, g.nz, P);
                if (s >= 0) {
                    const int o = (int)(g.psi_off[2] + 2 * g.slab[2]) + x + g.nx * (y + g.ny * s);
                    const int sl = (int)g.slab[2];
                    const float b = bE[s], a = aE[s], kv = kE[s];
                    const float p1 = b * psiE[o] + a * t1;
                    const float p2 = b * psiE[o + sl] + a * t2;
                    psiE[o] = p1;
                    psiE[o + sl] = p2;
                    t1 = kv * t1 + p1;
                    t2 = kv * t2 + p2;
                }
            }
            float ux = t0 - t1, uy = t2 - t3, uz = t4 - t5;
            if (in_box(x, y, k, g.src_lo, g.src_hi)) {
                const int sxn = g.src_hi[0] - g.src_lo[0], syn = g.src_hi[1] - g.src_lo[1];
                const float jv = wave * g.src_profile[(x - g.src_lo[0]) + sxn * ((y - g.src_lo[1]) + syn * (k - g.src_lo[2]))];
                if (g.src_comp == 0) ux -= jv; else if (g.src_comp == 1) uy -= jv; else uz -= jv;
            }
            const float c = g.dt / eps[idx];
            const float ex = sE[cur][0][row + 1][lane + 1] + c * ux;
            const float ey = sE[cur][1][row + 1][lane + 1] + c * uy;
            const float ez = sE[cur][2][row + 1][lane + 1] + c * uz;
            E1[idx] = ex;
            E1[N + idx] = ey;
            E1[2 * N + idx] = ez;
            if (in_box(x, y, k, g.det_lo, g.det_hi)) e2 += (double)ex * ex + (double)ey * ey + (double)ez * ez;
        }
        hx_prev = hx;
        hy_prev = hy;
        cur = nxt;
    }
    // detector partial of this tile (tiles intersecting the detector only; uniform per block)
    const int dx = tix - tl.dtx0, dy = tiy - tl.dty0, dz = tiz - tl.dtz0;
    if (dx < 0 || dy < 0 || dz < 0 || dx >= tl.dntx || dy >= tl.dnty || dz >= tl.dntz) return;
    for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off, 64);
    if (lane == 0) red[row] = e2;
    __syncthreads();
    if (tid == 0) {
        double sum = 0.0;
        for (int w = 0; w < TY; ++w) sum += red[w];
        partials[dx + (long long)tl.dntx * (dy + (long long)tl.dnty * dz)] = sum;
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

void launch_fwd_step(const Grid& g, const Tiling& t, const float* E0, const float* H0, float* E1, float* H1,
                     const float* psiH0, float* psiH1, float* psiE, const float* eps, float wave, double* partials,
                     void* store, float* staging, int slice, hipStream_t s) {
    if (t.ty == 8)
        launch_kernel(K_FWD_STEP, k_fwd_step<8>, dim3(t.count), dim3(TX, 8), s, g, t, E0, H0, E1, H1, psiH0, psiH1,
                      psiE, eps, wave, partials, store, staging, slice);
    else
        launch_kernel(K_FWD_STEP, k_fwd_step<4>, dim3(t.count), dim3(TX, 4), s, g, t, E0, H0, E1, H1, psiH0, psiH1,
                      psiE, eps, wave, partials, store, staging, slice);
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
