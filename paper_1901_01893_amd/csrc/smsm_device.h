// Device-side helpers for the SMS-MUSSELS kernels: complex double arithmetic,
// block reductions and a batched in-LDS radix-2 FFT.
//
// All arithmetic is FP64.  Complex numbers are double2 (re, im).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SMSM_DEV __device__ __forceinline__
#define SMSM_HD __host__ __device__

SMSM_DEV double2 cmk(double re, double im) { return make_double2(re, im); }
SMSM_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
SMSM_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
SMSM_DEV double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
SMSM_DEV double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
SMSM_DEV double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
SMSM_DEV double2 cmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
SMSM_DEV double2 cconjmul(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc + a * b
SMSM_DEV double2 cfma(double2 a, double2 b, double2 acc) {
    return make_double2(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}
SMSM_DEV double2 c64to128(float2 v) { return make_double2((double)v.x, (double)v.y); }
SMSM_DEV double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// (-1)^k as a double
SMSM_DEV double sgn_pow(int k) { return (k & 1) ? -1.0 : 1.0; }

// Sum of one double over the block, in a fixed order (deterministic).
// `scratch` must hold blockDim.x/64 doubles of shared memory.  Every thread
// must call it; the result is valid in all threads.
SMSM_DEV double block_sum(double v, double* scratch) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, warp = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[warp] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += scratch[w];
    __syncthreads();
    return s;
}

// N block sums with one exchange through shared memory (scratch: N *
// blockDim.x/64 doubles).  Every thread must call it; results in all threads.
template <int N>
SMSM_DEV void block_sum_n(double (&v)[N], double* scratch) {
#pragma unroll
    for (int k = 0; k < N; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    const int lane = threadIdx.x & 63, warp = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) scratch[k * nw + warp] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += scratch[k * nw + w];
        v[k] = s;
    }
    __syncthreads();
}

// Sum of `n` partial values in a fixed order (each thread of the block gets
// the same result).  Used to turn per-block partials into a scalar.  A thread
// adds its slots threadIdx.x + k blockDim.x in increasing k, loading eight
// slots at a time so they are in flight together.
SMSM_DEV double sum_partials(const double* __restrict__ part, int n, double* scratch) {
    const int nt = blockDim.x;
    double v = 0.0;
    for (int base = threadIdx.x; base < n; base += 8 * nt) {
        double pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = base + u * nt;
            pv[u] = part[k < n ? k : n - 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (base + u * nt < n) v += pv[u];
    }
    return block_sum(v, scratch);
}

// Sum of `n` partial values by one wave, in a fixed order (every lane, and
// every wave that calls it on the same data, gets the same result): lane
// adds slots lane + 64 k in increasing k, eight loads in flight, then a
// butterfly across the lanes (IEEE addition is commutative, so the partners
// of each step form identical sums).
SMSM_DEV double wave_sum_partials(const double* __restrict__ part, int n, int lane) {
    double v = 0.0;
    for (int base = lane; base < n; base += 8 * 64) {
        double pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = base + u * 64;
            pv[u] = part[k < n ? k : n - 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (base + u * 64 < n) v += pv[u];
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sums of two ranges of per-block partials, a[0..na) and b[0..nb), each in
// a fixed order (deterministic), with every load of a thread issued before the
// first add (8 slots per range per pass).  Every thread must call it; the
// results are valid in all threads.  scratch: 2 * blockDim.x/64 doubles.
SMSM_DEV void sum_partials2(const double* __restrict__ a, int na, const double* __restrict__ b, int nb,
                            double& sa, double& sb, double* scratch) {
    const int nt = blockDim.x, n = na > nb ? na : nb;
    double ta = 0.0, tb = 0.0;
    for (int base = threadIdx.x; base < n; base += 8 * nt) {
        double va[8], vb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = base + u * nt;
            va[u] = a[k < na ? k : na - 1];
            vb[u] = b[k < nb ? k : nb - 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = base + u * nt;
            ta += k < na ? va[u] : 0.0;
            tb += k < nb ? vb[u] : 0.0;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        ta += __shfl_xor(ta, off);
        tb += __shfl_xor(tb, off);
    }
    const int lane = threadIdx.x & 63, warp = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) {
        scratch[warp] = ta;
        scratch[nw + warp] = tb;
    }
    __syncthreads();
    sa = 0.0;
    sb = 0.0;
    for (int w = 0; w < nw; ++w) {
        sa += scratch[w];
        sb += scratch[nw + w];
    }
    __syncthreads();
}

// v mod n for v in [-n, 2n) (one wrap either way), any length n > 0.
SMSM_DEV int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// v mod n in [0, n) for any v (a mask when n is a power of two).
SMSM_DEV int imod(int v, int n) {
    if ((n & (n - 1)) == 0) return v & (n - 1);
    const int m = v % n;
    return m < 0 ? m + n : m;
}

// Outputs per thread of the final step of a transform whose length has an
// odd factor (each launch keeps nb n <= FFT_MIX_PER_THREAD x threads).
#define FFT_MIX_PER_THREAD 16

// Batched in-place FFT in shared memory.
// nb sequences of length n = q 2^logn (q = 1, or an odd factor such as 3 or
// 7); sequence b occupies buf[b*stride + j].  Forward computes
// X[k] = sum_j x[j] e^{-2 pi i jk/n}; inverse uses e^{+...} (both
// unnormalised).  tw[k] = e^{-2 pi i k/n}, k < n/2 for q = 1, k < n otherwise
// (global or shared).  For q > 1, decimation in time over the odd factor: the
// q interleaved sequences x[q m + r] (m < 2^logn) are transformed in place by
// the radix-2 stages, then X[k] = sum_{r<q} w_n^{r k} Y_r[k mod 2^logn] is
// formed in registers (at most FFT_MIX_PER_THREAD outputs per thread) and
// written back.  All threads of the block must call it; it starts and ends
// with a barrier.
// Exact division of 0 <= x by a runtime divisor 1 <= d with x d < 2^32 (here
// both stay below 2^16): q = floor(x m / 2^32) with m = ceil(2^32 / d), whose
// excess over 2^32 / d is below 1, so x m / 2^32 exceeds x / d by less than
// 1 / d and the floor is exact.  One high multiply per division.
struct FastDiv {
    unsigned d, m;
    SMSM_DEV explicit FastDiv(int dd) : d((unsigned)dd), m(dd > 1 ? 0xFFFFFFFFu / (unsigned)dd + 1u : 0u) {}
    SMSM_DEV int div(int x) const { return d > 1 ? (int)__umulhi((unsigned)x, m) : x; }
};

template <int NOUT = FFT_MIX_PER_THREAD>   // outputs per thread of the odd-factor step (nb n <= NOUT x threads)
SMSM_DEV void fft_batch_lds(double2* buf, int n, int logn, int nb, int stride,
                            const double2* __restrict__ tw, bool inverse) {
    const int tid = threadIdx.x, nt = blockDim.x;
    __syncthreads();
    const int q = n >> logn;
    if (q > 1) {
        const int p = 1 << logn, hp = p >> 1;
        const FastDiv fn(n), fq(q), fqh(q * hp);   // nb n stays below 2^16 (the register bound above)
        for (int idx = tid; idx < nb * n; idx += nt) {
            const int b = fn.div(idx), jj = idx - b * n, m = fq.div(jj), r = jj - m * q;
            const int rm = logn ? (int)(__brev((unsigned)m) >> (32 - logn)) : 0;
            if (m < rm) {
                double2* s = buf + b * stride;
                const double2 t = s[q * m + r];
                s[q * m + r] = s[q * rm + r];
                s[q * rm + r] = t;
            }
        }
        __syncthreads();
        for (int st = 0; st < logn; ++st) {
            const int half = 1 << st;
            for (int idx = tid; idx < nb * q * hp; idx += nt) {
                const int b = fqh.div(idx), rem = idx - b * q * hp, r = rem >> (logn - 1), k = rem & (hp - 1);
                const int pos = k & (half - 1);
                const int i0 = ((k >> st) << (st + 1)) + pos, i1 = i0 + half;
                double2 w = tw[(pos << (logn - 1 - st)) * q];   // w_p^(.) = w_n^(q .)
                if (inverse) w.y = -w.y;
                double2* base = buf + b * stride;
                const double2 a = base[q * i0 + r];
                const double2 c = cmul(base[q * i1 + r], w);
                base[q * i0 + r] = cadd(a, c);
                base[q * i1 + r] = csub(a, c);
            }
            __syncthreads();
        }
        double2 out[NOUT];
#pragma unroll
        for (int u = 0; u < NOUT; ++u) {
            const int idx = tid + u * nt;
            if (idx < nb * n) {
                const int b = fn.div(idx), k = idx - b * n, km = k & (p - 1);
                const double2* base = buf + b * stride + q * km;
                double2 acc = base[0];
                int ph = 0;                                   // r k mod n
                for (int r = 1; r < q; ++r) {
                    ph += k;
                    if (ph >= n) ph -= n;
                    double2 w = tw[ph];
                    if (inverse) w.y = -w.y;
                    acc = cfma(base[r], w, acc);
                }
                out[u] = acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NOUT; ++u) {
            const int idx = tid + u * nt;
            if (idx < nb * n) {
                const int b = fn.div(idx), k = idx - b * n;
                buf[b * stride + k] = out[u];
            }
        }
        __syncthreads();
        return;
    }
    if (logn == 0) return;
    for (int idx = tid; idx < nb * n; idx += nt) {
        const int b = idx >> logn, j = idx & (n - 1);
        const int rj = (int)(__brev((unsigned)j) >> (32 - logn));
        if (j < rj) {
            double2* s = buf + b * stride;
            const double2 t = s[j];
            s[j] = s[rj];
            s[rj] = t;
        }
    }
    __syncthreads();
    const int hn = n >> 1;
    for (int s = 0; s < logn; ++s) {
        const int half = 1 << s;
        for (int idx = tid; idx < nb * hn; idx += nt) {
            const int b = idx >> (logn - 1), k = idx & (hn - 1);
            const int pos = k & (half - 1);
            const int i0 = ((k >> s) << (s + 1)) + pos;
            const int i1 = i0 + half;
            double2 w = tw[pos << (logn - 1 - s)];
            if (inverse) w.y = -w.y;
            double2* base = buf + b * stride;
            const double2 a = base[i0];
            const double2 c = cmul(base[i1], w);
            base[i0] = cadd(a, c);
            base[i1] = csub(a, c);
        }
        __syncthreads();
    }
}
