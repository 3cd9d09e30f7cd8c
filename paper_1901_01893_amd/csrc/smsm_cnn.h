// Learned unrolled solver (an extension beyond the paper: a learned prior in
// place of the Hankel IRLS step).  Each unrolled iteration is
//   z = x + s C(x / s),   x <- (A^H A + mu I)^-1 (A^H y + mu z),
// C a real CNN over the 2 Ns channels (real and imaginary part of each shot's
// k-space) of every slice: five 3 x 3 layers with ReLU after the first four;
// s = sqrt(mean |A^H y|^2).  The network runs with FP32 weights on the
// vector ALU or with BF16 weights on the matrix cores (smsm_cnn_mfma.h), FP32
// accumulation and a fixed summation order either way; the data-consistency
// solves run in FP64 on the solver's normal operator.
//
// Layouts: activations [N][C][H][W] float (N = slices), weights
// [Co][Ci][3][3] then bias [Co] per layer, layers back to back.
#pragma once
#include "smsm_device.h"

#define CNN_THREADS 256
#define CNN_CONST __attribute__((address_space(4)))

// 3 x 3 convolution, zero padding, cross-correlation.  Forward (BWD = 0):
//   out[n][o][i][j] = bias[o] + sum_c sum_{a,d} w[o][c][a][d] in[n][c][i+a-1][j+d-1]
// (ReLU applied when relu != 0).  Backward data (BWD = 1), the transpose:
//   out[n][c][i][j] = sum_o sum_{a,d} w[o][c][2-a][2-d] in[n][o][i+a-1][j+d-1]
// with `in` the gradient of the layer output, ci = the layer's Co and co = its
// Ci here.  One thread per pixel and COB consecutive output channels; the
// weights of a (channel block, input channel) are wave-uniform and read
// through the scalar cache.  Sums run over input channels, then taps (row
// major), in order.  grid (ceil(H W / 256), co / COB, N), block 256.  (The
// network's BF16-weight form runs on the matrix cores: smsm_cnn_mfma.h.)
template <int COB, int BWD>
__global__ void __launch_bounds__(CNN_THREADS)
k_conv3x3(int ci, int co, int H, int W, const float* __restrict__ in, const float* __restrict__ wv,
          const float* __restrict__ bias, float* __restrict__ out, int relu) {
    const int npx = H * W;
    const int p = blockIdx.x * CNN_THREADS + threadIdx.x;
    const int o0 = blockIdx.y * COB, n = blockIdx.z;
    const bool live = p < npx;
    const int pp = live ? p : 0;
    const int i = pp / W, j = pp - i * W;
    float acc[COB];
#pragma unroll
    for (int u = 0; u < COB; ++u) acc[u] = (BWD || bias == nullptr) ? 0.0f : bias[o0 + u];
    const float* src = in + (size_t)n * ci * npx;
    for (int c = 0; c < ci; ++c) {
        float v[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int ii = i + a - 1, jj = j + d - 1;
                const bool in_b = ii >= 0 && ii < H && jj >= 0 && jj < W;
                v[3 * a + d] = in_b ? src[(size_t)c * npx + ii * W + jj] : 0.0f;
            }
#pragma unroll
        for (int u = 0; u < COB; ++u) {
            // forward: w[o0+u][c][t]; backward: w[c][o0+u][8-t]
            const size_t wo = BWD ? ((size_t)c * co + o0 + u) * 9 : ((size_t)(o0 + u) * ci + c) * 9;
            const CNN_CONST float* wp = (const CNN_CONST float*)(uintptr_t)(wv + wo);
#pragma unroll
            for (int t = 0; t < 9; ++t) acc[u] = fmaf(wp[BWD ? 8 - t : t], v[t], acc[u]);
        }
    }
    if (live) {
#pragma unroll
        for (int u = 0; u < COB; ++u) {
            const float r = (relu && acc[u] < 0.0f) ? 0.0f : acc[u];
            out[((size_t)n * co + o0 + u) * npx + p] = r;
        }
    }
}

// Weight and bias gradients of one layer: for the block's (o, c)
//   gw[o][c][a][d] (+)= sum_{n,i,j} gout[n][o][i][j] in[n][c][i+a-1][j+d-1],
//   gb[o] (+)= sum_{n,i,j} gout[n][o][i][j]   (blocks with c = 0).
// Thread t takes pixels t, t + 256, ... of each image in order; the block
// sums the thread partials in a fixed order (deterministic).  accumulate
// adds to the existing gradient (weights shared across iterations).
// grid (Ci * Co), block 256; block b -> o = b / Ci, c = b % Ci.
__global__ void __launch_bounds__(CNN_THREADS)
k_conv3x3_wgrad(int N, int ci, int co, int H, int W, const float* __restrict__ in, const float* __restrict__ gout,
                float* __restrict__ gw, float* __restrict__ gb, int accumulate) {
    __shared__ float red[10][CNN_THREADS / 64];
    const int o = blockIdx.x / ci, c = blockIdx.x - o * ci;
    const int npx = H * W;
    float acc[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) acc[t] = 0.0f;
    for (int n = 0; n < N; ++n) {
        const float* g = gout + ((size_t)n * co + o) * npx;
        const float* x = in + ((size_t)n * ci + c) * npx;
        for (int p = threadIdx.x; p < npx; p += CNN_THREADS) {
            const int i = p / W, j = p - i * W;
            const float gv = g[p];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int ii = i + a - 1, jj = j + d - 1;
                    const bool in_b = ii >= 0 && ii < H && jj >= 0 && jj < W;
                    acc[3 * a + d] = fmaf(gv, in_b ? x[ii * W + jj] : 0.0f, acc[3 * a + d]);
                }
            acc[9] += gv;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < 10; ++t) {
        float v = acc[t];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[t][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        const int t = threadIdx.x;
        float s = 0.0f;
        for (int k = 0; k < CNN_THREADS / 64; ++k) s += red[t][k];
        if (t < 9) {
            float* dst = gw + ((size_t)o * ci + c) * 9 + t;
            *dst = accumulate ? *dst + s : s;
        } else if (c == 0) {
            gb[o] = accumulate ? gb[o] + s : s;
        }
    }
}

// g[k] = 0 where the layer's ReLU output act[k] is 0 (gradient of the ReLU).
__global__ void k_relu_bwd(long n, float* __restrict__ g, const float* __restrict__ act) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        if (!(act[k] > 0.0f)) g[k] = 0.0f;
}

// Complex k-space [L][Ns][npx] (FP64) -> channels [L][2 Ns][npx] (FP32):
// channel 2i = f Re x_i, 2i + 1 = f Im x_i with f = 1 / *s (inv) or *s
// (1 / 0 taken as 0: all-zero data, where the prior's term s C(.) is 0).
__global__ void k_cnn_pack(long L, int ns, int npx, const double2* __restrict__ x, const double* __restrict__ s,
                           int inv, float* __restrict__ out) {
    const double sv = *s, f = inv ? (sv > 0.0 ? 1.0 / sv : 0.0) : sv;
    const long total = L * ns * npx;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long li = k / npx;            // l * ns + i
        const int p = (int)(k - li * npx);
        const double2 v = x[k];
        out[(2 * li) * npx + p] = (float)(v.x * f);
        out[(2 * li + 1) * npx + p] = (float)(v.y * f);
    }
}

// z = x + f (c_{2i} + i c_{2i+1}), f = 1 / *s (inv) or *s (1 / 0 taken as 0).
__global__ void k_cnn_unpack_add(long L, int ns, int npx, const float* __restrict__ c, const double2* __restrict__ x,
                                 const double* __restrict__ s, int inv, double2* __restrict__ z) {
    const double sv = *s, f = inv ? (sv > 0.0 ? 1.0 / sv : 0.0) : sv;
    const long total = L * ns * npx;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long li = k / npx;
        const int p = (int)(k - li * npx);
        const double2 v = x[k];
        z[k] = make_double2(v.x + f * (double)c[(2 * li) * npx + p], v.y + f * (double)c[(2 * li + 1) * npx + p]);
    }
}

// Adam on FP32 parameters: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void k_adam(long n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const float gk = g[k];
        const float mk = b1 * m[k] + (1.0f - b1) * gk;
        const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
        m[k] = mk;
        v[k] = vk;
        w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    }
}

// Vector helpers of the data-consistency CG (natural layout, FP64).
// out = a + f b, or f b when a is null (f = *fp * fm, or fm when fp is null).
// out may be a or b (each element is read before it is written).
__global__ void k_dc_axpy(long n, const double2* a, const double2* b, const double* __restrict__ fp, double fm,
                          double2* out) {
    const double f = fp ? *fp * fm : fm;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        out[k] = a ? cadd(a[k], cscale(b[k], f)) : cscale(b[k], f);
}

// Per-block partials of Re <a, b>.
__global__ void k_dc_dot(long n, const double2* __restrict__ a, const double2* __restrict__ b,
                         double* __restrict__ part) {
    __shared__ double red[16];
    double s = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const double2 u = a[k], v = b[k];
        s += u.x * v.x + u.y * v.y;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// One-block scalar step of the data-consistency CG from the partials:
//   mode 0: out[0] = sum(pa)                         (|r|^2)
//   mode 1: out[0] = *rr / sum(pa)                   (alpha = rr / <p, M p>; 0 if rr = 0)
//   mode 2: out[0] = sum(pa) / *rr, then *rr = sum(pa)   (beta; |r|^2 advanced)
//   mode 3: out[0] = sqrt(sum(pa) / count)           (data scale)
__global__ void k_dc_scalar(int mode, const double* __restrict__ pa, int np, double* rr, double count,
                            double* out) {
    __shared__ double red[16];
    const double s = sum_partials(pa, np, red);
    if (threadIdx.x == 0) {
        if (mode == 0) {
            out[0] = s;
        } else if (mode == 1) {
            const double r = *rr;
            out[0] = (r > 0.0 && s > 0.0) ? r / s : 0.0;
        } else if (mode == 2) {
            const double r = *rr;
            out[0] = r > 0.0 ? s / r : 0.0;
            *rr = s;
        } else {
            out[0] = sqrt(s / count);
        }
    }
}

// Fused steps of the data-consistency CG (the same arithmetic, in the same
// order, as k_dc_axpy / k_dc_dot / k_dc_scalar taken one after another, on
// the same grid, so the results are the same to the bit):
// q += mu p (the regularised normal operator) and per-block partials of
// Re <p, q>.
__global__ void k_dc_qdot(long n, const double2* __restrict__ p, double2* __restrict__ q, double mu,
                          double* __restrict__ part) {
    __shared__ double red[16];
    double s = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const double2 u = p[k], v = cadd(q[k], cscale(u, mu));
        q[k] = v;
        s += u.x * v.x + u.y * v.y;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}
// alpha = rr / sum(part_pq) (0 unless both are positive; every block forms it
// from the partials), x += alpha p, r -= alpha q, per-block partials of |r|^2.
__global__ void k_dc_xr(long n, double2* __restrict__ x, double2* __restrict__ r, const double2* __restrict__ p,
                        const double2* __restrict__ q, const double* __restrict__ part_pq, int np,
                        const double* __restrict__ rr, double* __restrict__ part_rr) {
    __shared__ double red[16];
    const double pq = sum_partials(part_pq, np, red), r0 = *rr;
    const double alpha = (r0 > 0.0 && pq > 0.0) ? r0 / pq : 0.0;
    double s = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        x[k] = cadd(x[k], cscale(p[k], alpha * 1.0));
        const double2 v = cadd(r[k], cscale(q[k], alpha * -1.0));
        r[k] = v;
        s += v.x * v.x + v.y * v.y;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
}
// rr_new = sum(part_rr), beta = rr_new / *rr_cur (0 when *rr_cur is 0),
// p = r + beta p; block 0 stores rr_new in *rr_next (a different slot from
// rr_cur, which the other blocks still read).
__global__ void k_dc_p(long n, const double2* __restrict__ r, double2* __restrict__ p,
                       const double* __restrict__ part_rr, int np, const double* __restrict__ rr_cur,
                       double* __restrict__ rr_next) {
    __shared__ double red[16];
    const double s = sum_partials(part_rr, np, red), r0 = *rr_cur;
    const double beta = r0 > 0.0 ? s / r0 : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *rr_next = s;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        p[k] = cadd(r[k], cscale(p[k], beta * 1.0));
}

// g = 2 g / *den (the loss gradient 2 (x - xt) / ||xt||^2 from g = x - xt).
__global__ void k_dc_grad0(long n, double2* __restrict__ g, const double* __restrict__ den) {
    const double f = 2.0 / *den;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        g[k] = cscale(g[k], f);
}

// Per-block partials of |ax - y|^2 (ax FP64, y the complex64 measurement).
__global__ void k_dc_resid(long n, const double2* __restrict__ ax, const float2* __restrict__ y,
                           double* __restrict__ part) {
    __shared__ double red[16];
    double s = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const double dx = ax[k].x - (double)y[k].x, dy = ax[k].y - (double)y[k].y;
        s += dx * dx + dy * dy;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Weight gradients in two deterministic stages for channel counts that are
// multiples of 8.  Stage 1: one workgroup per (pixel chunk, 8 output
// channels, 8 input channels); a chunk is WG_ROWS(W) whole rows of one image
// (WG_PX pixels).  The chunk's output gradients and its input rows with a
// one-pixel zero halo are staged in shared memory; thread (wave w, lane) owns
// the pair o = lane / 8, c = lane % 8 and its 9 taps over the w-th quarter of
// the chunk's pixels, taken in order with the 3 x 3 input window slid along
// the row (one gradient and three input reads per pixel; the 64 lanes of a
// wave read the same pixel: shared-memory broadcasts); the 4 waves' sums are
// added in order and stored as
//   part[chunk][o][c][t]   and, for the first input-channel block, the
//   bias partials bpart[chunk][o].
// Stage 2 (k_wgrad_sum) adds the chunks in order.
#define WG_PX 512
#define WG_TILE 8
__host__ __device__ inline int wg_rows(int H, int W) {
    const int r = WG_PX / W;
    return r < 1 ? 1 : (r > H ? H : r);
}
__host__ __device__ inline int wg_chunks(int H, int W) {
    const int r = wg_rows(H, W);
    return (H + r - 1) / r;
}
// staged input floats per channel: (rows + 2) x (W + 2); W <= 256
#define WG_IN_MAX (((WG_PX / 256) + 2) * 258 > 34 * 34 ? ((WG_PX / 256) + 2) * 258 : 34 * 34)

__global__ void __launch_bounds__(CNN_THREADS)
k_wgrad_part(int ci, int co, int H, int W, const float* __restrict__ in, const float* __restrict__ gout,
             float* __restrict__ part, float* __restrict__ bpart) {
    __shared__ float gs[WG_TILE][WG_PX];
    __shared__ float xs[WG_TILE][WG_IN_MAX];
    __shared__ float red[4][64][10];
    const int R = wg_rows(H, W), nch = wg_chunks(H, W);
    const int chunk = blockIdx.x, n = chunk / nch, r0 = (chunk - n * nch) * R;
    const int rows = (r0 + R <= H) ? R : H - r0;
    const int o0 = blockIdx.y * WG_TILE, c0 = blockIdx.z * WG_TILE;
    const int npx = H * W, W2 = W + 2;
    const int lw = __builtin_ctz((unsigned)W);        // W is a power of two
    const int tid = threadIdx.x;
    // stage: gout rows r0 .. r0 + rows - 1 of the 8 output channels (all
    // loads of a thread issued before its stores)
    {
        constexpr int NG = WG_TILE * WG_PX / CNN_THREADS;
        float v[NG];
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            const int k = tid + u * CNN_THREADS, o = k / WG_PX, q = k - o * WG_PX;
            v[u] = q < rows * W ? gout[((size_t)n * co + o0 + o) * npx + r0 * W + q] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            const int k = tid + u * CNN_THREADS, o = k / WG_PX, q = k - o * WG_PX;
            if (q < R * W) gs[o][q] = v[u];
        }
    }
    // stage: input rows r0 - 1 .. r0 + rows with a zero halo, 8 input
    // channels.  Flat index k -> (channel, row, column) by multiply-high with
    // ceil(2^32 / d): exact for k < 2^32 / d (here k < 8 * 34 * 34, d <= 258).
    {
        const int S = (R + 2) * W2;
        const unsigned mS = 0xFFFFFFFFu / (unsigned)S + 1u, mW = 0xFFFFFFFFu / (unsigned)W2 + 1u;
        constexpr int NX = (WG_TILE * WG_IN_MAX + CNN_THREADS - 1) / CNN_THREADS;
        float v[NX];
#pragma unroll
        for (int u = 0; u < NX; ++u) {
            const unsigned k = tid + u * CNN_THREADS;
            const int c = (int)__umulhi(k, mS), q = (int)k - c * S;
            const int rr = (int)__umulhi((unsigned)q, mW), jj = q - rr * W2;
            const int i = r0 - 1 + rr, j = jj - 1;
            const bool ok = c < WG_TILE && i >= 0 && i < H && j >= 0 && j < W;
            v[u] = ok ? in[((size_t)n * ci + c0 + c) * npx + i * W + j] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < NX; ++u) {
            const unsigned k = tid + u * CNN_THREADS;
            const int c = (int)__umulhi(k, mS), q = (int)k - c * S;
            if (c < WG_TILE) xs[c][q] = v[u];
        }
    }
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    const int o = lane >> 3, c = lane & 7;
    float acc[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) acc[t] = 0.0f;
    const int P = rows * W, qb = (P * w) / 4, qe = (P * (w + 1)) / 4;
    float win[3][3];
    for (int q = qb; q < qe; ++q) {
        const int i = q >> lw, j = q & (W - 1);
        const float* xp = &xs[c][i * W2 + j];          // top-left of the 3 x 3 window
        if (q == qb || j == 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int d = 0; d < 3; ++d) win[a][d] = xp[a * W2 + d];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                win[a][0] = win[a][1];
                win[a][1] = win[a][2];
                win[a][2] = xp[a * W2 + 2];
            }
        }
        const float gv = gs[o][q];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int d = 0; d < 3; ++d) acc[3 * a + d] = fmaf(gv, win[a][d], acc[3 * a + d]);
        acc[9] += gv;
    }
#pragma unroll
    for (int t = 0; t < 10; ++t) red[w][lane][t] = acc[t];
    __syncthreads();
    for (int k = tid; k < 64 * 10; k += CNN_THREADS) {
        const int pl = k / 10, t = k - pl * 10;
        const float s = ((red[0][pl][t] + red[1][pl][t]) + red[2][pl][t]) + red[3][pl][t];
        const int oo = pl >> 3, cc = pl & 7;
        if (t < 9) part[(((size_t)chunk * co + o0 + oo) * ci + c0 + cc) * 9 + t] = s;
        else if (blockIdx.z == 0 && cc == 0) bpart[(size_t)chunk * co + o0 + oo] = s;
    }
}

// gw[o][c][t] (+)= sum over chunks of part[chunk][o][c][t];
// gb[o] (+)= sum of bpart[chunk][o].  Block (WGS_OUT, WGS_SLICES): thread
// (x, y) adds, in chunk order, the chunks of slice y (consecutive runs of
// ceil(nchunk / WGS_SLICES)) for output blockIdx.x WGS_OUT + x, so that its
// loads are in flight together; the slice sums are then added in slice
// order.  The order is fixed, so the result is deterministic.
#define WGS_OUT 64
#define WGS_SLICES 16
__global__ void __launch_bounds__(WGS_OUT * WGS_SLICES)
k_wgrad_sum(int nchunk, int ci, int co, const float* __restrict__ part, const float* __restrict__ bpart,
            float* __restrict__ gw, float* __restrict__ gb, int accumulate) {
    __shared__ float red[WGS_SLICES][WGS_OUT];
    const int nw = co * ci * 9, x = threadIdx.x, y = threadIdx.y;
    const int k = blockIdx.x * WGS_OUT + x;
    const int per = (nchunk + WGS_SLICES - 1) / WGS_SLICES, c0 = y * per, c1 = min(c0 + per, nchunk);
    float s = 0.0f;
    if (k < nw) {
#pragma unroll 16
        for (int ch = c0; ch < c1; ++ch) s += part[(size_t)ch * nw + k];
    } else if (k < nw + co) {
        for (int ch = c0; ch < c1; ++ch) s += bpart[(size_t)ch * co + (k - nw)];
    }
    red[y][x] = s;
    __syncthreads();
    if (y == 0 && k < nw + co) {
        float t = red[0][x];
#pragma unroll
        for (int j = 1; j < WGS_SLICES; ++j) t += red[j][x];
        float* dst = k < nw ? gw + k : gb + (k - nw);
        *dst = accumulate ? *dst + t : t;
    }
}
