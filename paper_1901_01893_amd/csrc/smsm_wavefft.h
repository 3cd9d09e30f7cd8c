// In-wave FFTs of length N = 16..256 held in registers (FP64).
//
// N >= 64: one wave per sequence, lane j holds x[j + 64 t] for t < R = N/64.
// N <  64: groups of N lanes, one sequence per group, one value per lane.
// The transform is decimation in frequency: a radix-R stage on the values of
// a lane (with twiddles w_N^(j k1)), then log2(lanes) butterfly stages across
// lanes.  Output: the value at register k1 of lane j is X[k1 + R * brev(j)],
// brev over log2(lanes) bits.  `INV` selects the conjugate transform
// (unnormalised inverse).
#pragma once
#include "smsm_col_fast.h"

template <int N>
struct WaveFft {
    static constexpr int LANES = N >= 64 ? 64 : N;
    static constexpr int R = N >= 64 ? N / 64 : 1;
    static constexpr int LOGL = LANES == 64 ? 6 : LANES == 32 ? 5 : LANES == 16 ? 4 : LANES == 8 ? 3 : 2;
    double2 w[6];     // per-stage butterfly twiddle (1 on upper lanes)
    double sg[6];     // +1 upper lane, -1 lower lane
    double2 wr[3];    // radix-R stage twiddles w_N^(j k1), k1 = 1..R-1
    int m;            // lane index inside the sequence

    // tw: table of w_N^k = exp(-2 pi i k / N), k < N
    SMSM_DEV void setup(const double2* __restrict__ tw, int lane) {
        m = lane & (LANES - 1);
#pragma unroll
        for (int st = 0; st < LOGL; ++st) {
            const int h = 1 << st;
            const bool upper = (m & h) == 0;
            sg[st] = upper ? 1.0 : -1.0;
            w[st] = upper ? cmk(1.0, 0.0) : tw[(m & (h - 1)) * (LANES / (2 * h)) * R];
        }
#pragma unroll
        for (int k = 1; k < R; ++k) wr[k - 1] = tw[m * k];
    }

    // position of register k1 of this lane in the transformed sequence
    SMSM_DEV int out_index(int k1) const {
        const int br = (int)(__brev((unsigned)m) >> (32 - LOGL));
        return k1 + R * br;
    }

    template <bool INV>
    SMSM_DEV void run(double2 (&v)[R]) const {
        if constexpr (R == 4) {
            const double2 a = v[0], b = v[1], c = v[2], d = v[3];
            const double2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = csub(b, d);
            // forward: w_4 = -i ; inverse: +i
            const double2 jd1 = INV ? cmk(-d1.y, d1.x) : cmk(d1.y, -d1.x);
            v[0] = cadd(s0, s1);
            v[2] = csub(s0, s1);
            v[1] = cadd(d0, jd1);
            v[3] = csub(d0, jd1);
#pragma unroll
            for (int k = 1; k < 4; ++k) v[k] = cmul(v[k], INV ? cconj(wr[k - 1]) : wr[k - 1]);
        } else if constexpr (R == 2) {
            const double2 a = v[0], b = v[1];
            v[0] = cadd(a, b);
            v[1] = cmul(csub(a, b), INV ? cconj(wr[0]) : wr[0]);
        }
        if constexpr (LANES >= 64) dif_stage<32, R>(v, sg[5], INV ? cconj(w[5]) : w[5]);
        if constexpr (LANES >= 32) dif_stage<16, R>(v, sg[4], INV ? cconj(w[4]) : w[4]);
        if constexpr (LANES >= 16) dif_stage<8, R>(v, sg[3], INV ? cconj(w[3]) : w[3]);
        if constexpr (LANES >= 8) dif_stage<4, R>(v, sg[2], INV ? cconj(w[2]) : w[2]);
        dif_stage<2, R>(v, sg[1], INV ? cconj(w[1]) : w[1]);
        dif_stage<1, R>(v, sg[0], INV ? cconj(w[0]) : w[0]);
    }
};

// ---------------------------------------------------------------------------
// Row passes with in-wave FFTs.  A workgroup of 4 waves handles TR rows of one
// image b; each wave transforms whole rows in registers and parks them in a
// shared tile, which is then read out transposed (row pass 1) or staged from a
// transposed read (row pass 3), so global accesses stay coalesced.
// TR must be a multiple of (blockDim / 64) * (64 / LANES), and TR * N <= 8 * blockDim.
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(256)
k_rows_inv_w(Geo g, const double2* __restrict__ in, double2* __restrict__ out, const double2* __restrict__ tw1,
             int TR) {
    using F = WaveFft<N>;
    constexpr int R = F::R, LANES = F::LANES, G = 64 / LANES, ST = N + 1;
    extern __shared__ double2 sm[];
    const int b = blockIdx.y, j0 = blockIdx.x * TR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    F f;
    f.setup(tw1, lane);
    const int grp = lane / LANES;
    const size_t img = (size_t)b * g.n2 * N;
    const double sc = 1.0 / sqrt((double)N);
    for (int rb = 0; rb < TR; rb += nw * G) {
        const int r = rb + wave * G + grp;
        const size_t o = img + (size_t)(j0 + r) * N;
        double2 v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int k = f.m + 64 * t;
            v[t] = cscale(in[o + k], sgn_pow(k));
        }
        f.template run<true>(v);
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int n = f.out_index(t);
            sm[r * ST + n] = cscale(v[t], sc * sgn_pow(n));
        }
    }
    __syncthreads();
    const size_t ob = (size_t)b * N * g.n2;
    for (int idx = threadIdx.x; idx < TR * N; idx += blockDim.x) {
        const int c = idx / TR, jr = idx - c * TR;
        out[ob + (size_t)c * g.n2 + j0 + jr] = sm[jr * ST + c];
    }
}

template <int N>
__global__ void __launch_bounds__(256)
k_rows_fwd_w(Geo g, const double2* __restrict__ in, double2* __restrict__ out, const double2* __restrict__ tw1,
             int TR) {
    using F = WaveFft<N>;
    constexpr int R = F::R, LANES = F::LANES, G = 64 / LANES, ST = N + 1;
    extern __shared__ double2 sm[];
    const int b = blockIdx.y, j0 = blockIdx.x * TR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const size_t ib = (size_t)b * N * g.n2;
    for (int idx = threadIdx.x; idx < TR * N; idx += blockDim.x) {
        const int c = idx / TR, jr = idx - c * TR;
        sm[jr * ST + c] = in[ib + (size_t)c * g.n2 + j0 + jr];
    }
    __syncthreads();
    F f;
    f.setup(tw1, lane);
    const int grp = lane / LANES;
    const double sc = 1.0 / sqrt((double)N);
    for (int rb = 0; rb < TR; rb += nw * G) {
        const int r = rb + wave * G + grp;
        double2 v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int x = f.m + 64 * t;
            v[t] = cscale(sm[r * ST + x], sgn_pow(x));
        }
        f.template run<false>(v);
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int k = f.out_index(t);
            sm[r * ST + k] = cscale(v[t], sc * sgn_pow(k));
        }
    }
    __syncthreads();
    const size_t img = (size_t)b * g.n2 * N;
    for (int idx = threadIdx.x; idx < TR * N; idx += blockDim.x) {
        const int jr = idx / N, k = idx - jr * N;
        out[img + (size_t)(j0 + jr) * N + k] = sm[jr * ST + k];
    }
}

// ---------------------------------------------------------------------------
// Row passes for lengths with an odd factor (n1 = 3 or 7 times a power of
// two), which the in-wave forms do not take: TR rows of one image per
// workgroup, staged in shared memory (row stride n1 + 1) and transformed by
// fft_batch_lds.  Same conventions as k_rows_inv_w / k_rows_fwd_w:
//   INV:  natural [B][n2][n1] -> hybrid [B][n1][n2], centred unitary inverse DFT along kx;
//   !INV: hybrid [B][n1][n2] -> natural [B][n2][n1], centred unitary forward DFT along x.
// grid (n2 / TR, B); TR n1 <= FFT_MIX_PER_THREAD x threads.
// ---------------------------------------------------------------------------
template <bool INV>
__global__ void __launch_bounds__(256)
k_rows_any(Geo g, const double2* __restrict__ in, double2* __restrict__ out, const double2* __restrict__ tw1,
           int TR) {
    extern __shared__ double2 sm[];
    const int n1 = g.n1, n2 = g.n2, st = n1 + 1;
    const int b = blockIdx.y, j0 = blockIdx.x * TR;
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        if (INV) {
            const int jr = idx / n1, c = idx - jr * n1;
            sm[jr * st + c] = cscale(in[((size_t)b * n2 + j0 + jr) * n1 + c], sgn_pow(c));
        } else {
            const int c = idx / TR, jr = idx - c * TR;
            sm[jr * st + c] = cscale(in[((size_t)b * n1 + c) * n2 + j0 + jr], sgn_pow(c));
        }
    }
    fft_batch_lds(sm, n1, g.logn1, TR, st, tw1, INV);
    const double sc = 1.0 / sqrt((double)n1);
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        if (INV) {
            const int c = idx / TR, jr = idx - c * TR;
            out[((size_t)b * n1 + c) * n2 + j0 + jr] = cscale(sm[jr * st + c], sc * sgn_pow(c));
        } else {
            const int jr = idx / n1, k = idx - jr * n1;
            out[((size_t)b * n2 + j0 + jr) * n1 + k] = cscale(sm[jr * st + k], sc * sgn_pow(k));
        }
    }
}

// Root-sum-of-squares image (as k_sos_cols) for n2 with an odd factor: the
// Ns columns of slice l at x inverse-transformed in shared memory ([Ns][n2]
// and the twiddles), shots added in order.  grid (n1, L).
__global__ void __launch_bounds__(256) k_sos_any(Geo g, const double2* __restrict__ h,
                                                 const double2* __restrict__ tw2, double* __restrict__ out) {
    extern __shared__ double2 sm[];
    const int n1 = g.n1, n2 = g.n2, Ns = g.Ns;
    const int x = blockIdx.x, l = blockIdx.y;
    double2* TW = sm + Ns * n2;
    for (int k = threadIdx.x; k < n2; k += blockDim.x) TW[k] = tw2[k];
    for (int idx = threadIdx.x; idx < Ns * n2; idx += blockDim.x) {
        const int i = idx / n2, k = idx - i * n2;
        sm[idx] = cscale(h[((size_t)(l * Ns + i) * n1 + x) * n2 + k], sgn_pow(k));
    }
    fft_batch_lds(sm, n2, g.logn2, Ns, n2, TW, true);
    const double sc2 = 1.0 / (double)n2;
    for (int y = threadIdx.x; y < n2; y += blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < Ns; ++i) s += cabs2(sm[i * n2 + y]);
        out[((size_t)l * n2 + y) * n1 + x] = sqrt(s * sc2);
    }
}

// ---------------------------------------------------------------------------
// Root-sum-of-squares image of each slice (the per-shot images of the forward
// model combined over shots):
//   out[l][y][x] = sqrt(sum_i |u_{l,i}[y][x]|^2),
// u the centred unitary inverse DFT along ky of the hybrid rows
// h[l Ns + i][x][.] (the kx transform is already done).  grid (n1, L),
// block 64: lanes in groups of LANES = min(N, 64) points, one shot per group
// at a time; the groups' partial sums are added in group order.
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(64) k_sos_cols(Geo g, const double2* __restrict__ h,
                                                 const double2* __restrict__ tw2, double* __restrict__ out) {
    using F = WaveFft<N>;
    constexpr int R = F::R, LANES = F::LANES, G = 64 / LANES;
    __shared__ double part[G][N];
    const int x = blockIdx.x, l = blockIdx.y, lane = threadIdx.x;
    F f;
    f.setup(tw2, lane);
    const int grp = lane / LANES;
    const double sc = 1.0 / sqrt((double)N);
    double acc[R];
#pragma unroll
    for (int t = 0; t < R; ++t) acc[t] = 0.0;
    for (int i0 = 0; i0 < g.Ns; i0 += G) {
        const int i = i0 + grp;
        const double live = i < g.Ns ? 1.0 : 0.0;
        const size_t o = ((size_t)(l * g.Ns + min(i, g.Ns - 1)) * g.n1 + x) * N;
        double2 v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int k = f.m + 64 * t;
            v[t] = cscale(h[o + k], sgn_pow(k));
        }
        f.template run<true>(v);
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int n = f.out_index(t);
            acc[t] += live * cabs2(cscale(v[t], sc * sgn_pow(n)));
        }
    }
#pragma unroll
    for (int t = 0; t < R; ++t) part[grp][f.out_index(t)] = acc[t];
    __syncthreads();
    for (int y = lane; y < N; y += 64) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) s += part[q][y];
        out[((size_t)l * g.n2 + y) * g.n1 + x] = sqrt(s);
    }
}
