// Dense K x K complex matrix work of the IRLS weight step on FP64 matrix
// cores: the coupled Newton-Schulz iteration for (G + eps I)^(-1/2) and the
// repeated squaring that estimates lambda_max(G).
//
// Matrices are stored row-major with a padded stride KP (multiple of 16) and
// zeros outside the leading K x K block, so tiles need no bounds checks and
// products keep the padding zero.  Products are formed in full: the iterates
// are Hermitian only up to rounding, and forcing them Hermitian (mirroring a
// triangle, or taking (M + M^H)/2) destroys the convergence of the coupled
// iteration when G + eps I is ill-conditioned.
//
// A 16 x 16 tile C[i0:i0+16, j0:j0+16] = sum_k A[i][k] B[k][j] is built from
// v_mfma_f64_16x16x4f64: lane l supplies A[i0 + l%16][k0 + l/16] and
// B[k0 + l/16][j0 + l%16]; register v of lane l returns C[4 v + l/16][l%16].
// A complex product takes three real products per step of 4 (Gauss):
// T1 += (Ar + Ai) Br, T2 += Ar (Bi - Br), T3 += Ai (Br + Bi), then
// Cr = T1 - T3 and Ci = T1 + T2 (a quarter fewer MFMAs than the four-product
// form; the iterates are O(1), so the cancellation in Cr costs nothing at
// the 1e-10 convergence threshold).  The 4 waves of a workgroup split the
// inner dimension; their partial tiles are summed in a fixed order.
#pragma once
#include "smsm_device.h"

#define HT 16    // output tile edge
#define HW 4     // waves per tile

typedef double hd4 __attribute__((ext_vector_type(4)));

SMSM_HD inline int dense_stride(int K) { return (K + HT - 1) / HT * HT; }
SMSM_HD inline int dense_tiles(int K) {
    const int nt = dense_stride(K) / HT;
    return nt * nt;
}

enum { HG_NS = 0, HG_PAIR = 1, HG_NORM = 2 };

struct HgArgs {
    const double2* A0;
    const double2* B0;
    double2* C0;
    const double2* A1;      // HG_PAIR: second product, blockIdx.z odd
    const double2* B1;
    double2* C1;
    const int* done_cur;    // HG_NS / HG_PAIR: slice converged before this iteration
    int* done_next;         // HG_PAIR: convergence after this iteration
    int* last;              // HG_PAIR: buffer parity of the latest update
    int par;
    double tol2;            // HG_PAIR: squared tolerance on ||I - Z Y||_F
    const double* part_in;  // HG_PAIR: ||I - ZY||^2 partials; HG_NORM: ||P||^2 partials of the input
    int np_in;              // partials per slice in part_in
    double* part_out;       // HG_NS: |I - ZY|^2 partials; HG_NORM: |C|^2 partials (per tile)
    const double* mu;       // HG_NS: scale factor of this iteration, per slice (stride mu_stride)
    int mu_stride;
};

// Scaled coupled Newton-Schulz step.  With X = Z Y (spectrum in [lo, 1],
// a function of A, Y = (A/c) Z throughout), T = sqrt(mu) (1.5 I - 0.5 mu X)
// maps an eigenvalue x of X to f(mu x), f(x) = x (1.5 - 0.5 x)^2, which has
// its maximum 1 at x = 1.  For lo far below 1, mu in (1, NS_MU_MAX] is chosen
// so that f(mu lo) = f(mu) (both ends of the interval land at the same
// height), which raises the lower end about 5.6x per step instead of 2.25x;
// once lo > NS_MU_SWITCH the plain step (mu = 1) converges quadratically.
// NS_MU_MAX keeps mu x well below 3, where f turns negative, when rounding
// puts an eigenvalue slightly above 1.
#define NS_MU_MAX 2.5
#define NS_MU_SWITCH 0.3
SMSM_DEV double ns_f(double x) {
    const double t = 1.5 - 0.5 * x;
    return x * t * t;
}
// mu[k] for k < nit from the lower bound lo of the initial spectrum
SMSM_DEV void ns_schedule(double lo, int nit, double* mu, int stride) {
    for (int k = 0; k < nit; ++k) {
        double m = 1.0;
        if (lo <= NS_MU_SWITCH && lo * NS_MU_MAX < 1.0) {
            if (ns_f(NS_MU_MAX) - ns_f(NS_MU_MAX * lo) > 0.0) {
                m = NS_MU_MAX;
            } else {
                double a = 1.0, b = NS_MU_MAX;
                for (int it = 0; it < 60; ++it) {
                    const double c = 0.5 * (a + b);
                    if (ns_f(c) - ns_f(c * lo) > 0.0) a = c;
                    else b = c;
                }
                m = 0.5 * (a + b);
            }
            lo = fmin(ns_f(m * lo), ns_f(m));
        } else {
            lo = fmin(ns_f(lo), 1.0);
        }
        mu[(size_t)k * stride] = m;
    }
}

// MODE HG_NS  : C0 = sqrt(mu) (1.5 I - 0.5 mu A0 B0)   (T of the scaled iteration, A0 = Z, B0 = Y)
// MODE HG_PAIR: C0 = A0 B0, C1 = A1 B1        (Y T and T Z), grid z = 2 l + which
// MODE HG_NORM: C0 = A0 B0 / sum(part_in_l)   (normalised squaring, A0 = B0 = P)
// grid (dense_tiles(K), 1, L or 2L), block 64 * HW; tile t = bi * nt + bj.
template <int MODE>
__global__ void __launch_bounds__(64 * HW) k_zgemm(int K, int KP, HgArgs a) {
    __shared__ double acc[HW][8][64];
    __shared__ double red[16];
    const int z = blockIdx.z;
    const int l = MODE == HG_PAIR ? z >> 1 : z;
    const int which = MODE == HG_PAIR ? z & 1 : 0;
    const int ntile = gridDim.x;
    if (MODE != HG_NORM) {
        if (a.done_cur[l]) {
            if (MODE == HG_PAIR && blockIdx.x == 0 && which == 0 && threadIdx.x == 0) a.done_next[l] = 1;
            return;
        }
    }
    double sc = 1.0;
    if (MODE == HG_PAIR) {
        const double res2 = sum_partials(a.part_in + (size_t)l * a.np_in, a.np_in, red);
        if (blockIdx.x == 0 && which == 0 && threadIdx.x == 0) {
            a.done_next[l] = (res2 < a.tol2) ? 1 : 0;
            a.last[l] = a.par;
        }
    } else if (MODE == HG_NORM) {
        const double f = sum_partials(a.part_in + (size_t)l * a.np_in, a.np_in, red);
        sc = f > 0.0 ? 1.0 / f : 0.0;
    }
    const double2* A = which ? a.A1 : a.A0;
    const double2* B = which ? a.B1 : a.B0;
    double2* C = which ? a.C1 : a.C0;
    const size_t off = (size_t)l * KP * KP;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nt = KP / HT;
    const int bi = blockIdx.x / nt, bj = blockIdx.x - bi * nt;
    const int i0 = bi * HT, j0 = bj * HT;
    const int kq = lane >> 4;
    const double2* Ap = A + off + (size_t)(i0 + (lane & 15)) * KP + kq;   // A[i][kq + 4 s]
    const double2* Bp = B + off + (size_t)kq * KP + j0 + (lane & 15);     // B[kq + 4 s][j]
    const int nks = (K + 3) / 4;   // columns of A and rows of B past K are zero: skipped
    const int ks0 = (w * nks) / HW, ks1 = ((w + 1) * nks) / HW;
    hd4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = {0.0, 0.0, 0.0, 0.0}, t3 = {0.0, 0.0, 0.0, 0.0};
    int ks = ks0;
    // batches of 4 steps: all 8 loads issued before the 16 products
    for (; ks + 4 <= ks1; ks += 4) {
        double2 av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            av[u] = Ap[4 * (ks + u)];
            bv[u] = Bp[(size_t)4 * (ks + u) * KP];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x + av[u].y, bv[u].x, t1, 0, 0, 0);
            t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv[u].y - bv[u].x, t2, 0, 0, 0);
            t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].y, bv[u].x + bv[u].y, t3, 0, 0, 0);
        }
    }
    for (; ks < ks1; ++ks) {
        const double2 av = Ap[4 * ks], bv = Bp[(size_t)4 * ks * KP];
        t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x + av.y, bv.x, t1, 0, 0, 0);
        t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y - bv.x, t2, 0, 0, 0);
        t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x + bv.y, t3, 0, 0, 0);
    }
    const hd4 cr = t1 - t3, ci = t1 + t2;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        acc[w][v][lane] = cr[v];
        acc[w][4 + v][lane] = ci[v];
    }
    __syncthreads();
    const int v = threadIdx.x >> 6, ln = threadIdx.x & 63;
    double2 c = cmk(0.0, 0.0);
#pragma unroll
    for (int ww = 0; ww < HW; ++ww) {
        c.x += acc[ww][v][ln];
        c.y += acc[ww][4 + v][ln];
    }
    const int R = i0 + 4 * v + (ln >> 4), Cc = j0 + (ln & 15);
    double contrib = 0.0;
    if (MODE == HG_NS) {
        const double dl = (R == Cc && R < K) ? 1.0 : 0.0;
        contrib = (dl - c.x) * (dl - c.x) + c.y * c.y;
        const double mu = a.mu[(size_t)l * a.mu_stride], rm = sqrt(mu);
        c = cmk(rm * (1.5 * dl - 0.5 * mu * c.x), -0.5 * rm * mu * c.y);
    } else if (MODE == HG_NORM) {
        c = cscale(c, sc);
        contrib = cabs2(c);
    }
    C[off + (size_t)R * KP + Cc] = c;
    if (MODE != HG_PAIR) {
        const double s = block_sum(contrib, red);
        if (threadIdx.x == 0) a.part_out[(size_t)l * ntile + blockIdx.x] = s;
    }
}

// Out_l = Herm(G_l) + eps_l I in the padded layout (eps_l = mult * src[l], or
// 0 when src is null), Herm(M) = (M + M^H) / 2, and per-block partials of
// ||Out_l||_F^2.  grid (nblk, L).
__global__ void k_dense_pad(int K, int KP, const double2* __restrict__ G, const double* __restrict__ src,
                           double mult, double2* __restrict__ Out, double* __restrict__ part) {
    __shared__ double red[16];
    const int l = blockIdx.y;
    const double eps = src ? mult * src[l] : 0.0;
    const double2* Gl = G + (size_t)l * K * K;
    double s = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < KP * KP; idx += gridDim.x * blockDim.x) {
        const int i = idx / KP, j = idx - i * KP;
        double2 v = cmk(0.0, 0.0);
        if (i < K && j < K) {
            const double2 u = Gl[(size_t)i * K + j], t = Gl[(size_t)j * K + i];
            v = cmk(0.5 * (u.x + t.x), 0.5 * (u.y - t.y));
            if (i == j) v = cmk(v.x + eps, 0.0);
        }
        Out[(size_t)l * KP * KP + idx] = v;
        s += cabs2(v);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[(size_t)l * gridDim.x + blockIdx.x] = s;
}

// Start of the coupled Newton-Schulz iteration: Y = Out / c, Z = I with
// c = ||G + eps I||_F from the k_dense_pad partials.  eps_l <= 0 (or G = 0)
// marks slice l unregularised: done[l] = 1 and wscale_l = 0 (W_l = 0).
// Clears the flags done[1..nit] and the parity record, and writes the scale
// factors mu[k][l] of the scaled iteration.  grid (nblk, L).
__global__ void k_ns_start(int K, int KP, int L, const double* __restrict__ src, double mult,
                           const double* __restrict__ part, int np, double2* __restrict__ Y,
                           double2* __restrict__ Z, double* __restrict__ wscale, int* __restrict__ done, int nit,
                           double* __restrict__ mu) {
    __shared__ double red[16];
    const int l = blockIdx.y;
    const double eps = mult * src[l];
    const double fro2 = sum_partials(part + (size_t)l * np, np, red);
    const bool unreg = !(eps > 0.0) || !(fro2 > 0.0);
    const double ic = unreg ? 1.0 : 1.0 / sqrt(fro2);
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < KP * KP; idx += gridDim.x * blockDim.x) {
        const int i = idx / KP, j = idx - i * KP;
        const size_t o = (size_t)l * KP * KP + idx;
        Y[o] = cscale(Y[o], ic);
        Z[o] = cmk((i == j && i < K) ? 1.0 : 0.0, 0.0);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        wscale[l] = unreg ? 0.0 : sqrt(ic);
        done[l] = unreg ? 1 : 0;
        for (int k = 1; k <= nit; ++k) done[k * L + l] = 0;
        done[(nit + 1) * L + l] = 0;
        // spectrum of (G + eps I) / c lies in [eps / c, 1]
        ns_schedule(unreg ? 1.0 : eps * ic, nit, mu + l, L);
    }
}

// W_l = wscale_l * Z_l (unpadded K x K), Z_l from the buffer the last
// executed iteration wrote.
__global__ void k_ns_finish(int K, int KP, int L, const double2* __restrict__ Z0, const double2* __restrict__ Z1,
                            const int* __restrict__ last, const int* __restrict__ conv,
                            const double* __restrict__ wscale, double2* __restrict__ W, int* __restrict__ flags) {
    const long total = (long)L * K * K;
    const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int l = (int)(idx / ((long)K * K));
    const int rem = (int)(idx - (long)l * K * K);
    // conv[l]: slice l met the tolerance within the iteration cap (or is
    // unregularised); otherwise the plan's status word records it
    if (rem == 0 && !conv[l]) flags[1] = 1;
    const int i = rem / K, j = rem - i * K;
    const size_t o = (size_t)l * KP * KP + (size_t)i * KP + j;
    W[idx] = cscale((last[l] ? Z1 : Z0)[o], wscale[l]);
}

// Partials of Re tr(G P) and Re tr(P) for the Rayleigh quotient of the
// squared matrix P (padded); num partials at part[l * nblk + b], den partials
// at part[(L + l) * nblk + b].  grid (nblk, L).
__global__ void k_trace_part(int K, int KP, const double2* __restrict__ G, const double2* __restrict__ P,
                             double* __restrict__ part) {
    __shared__ double red[16];
    const int l = blockIdx.y, L = gridDim.y, nb = gridDim.x;
    const double2* Gl = G + (size_t)l * K * K;
    const double2* Pl = P + (size_t)l * KP * KP;
    double num = 0.0, den = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < K * K; idx += nb * blockDim.x) {
        const int j = idx / K, m = idx - j * K;
        const double2 gp = cmul(Gl[idx], Pl[(size_t)m * KP + j]);
        num += gp.x;
        if (j == m) den += Pl[(size_t)j * KP + j].x;
    }
    num = block_sum(num, red);
    den = block_sum(den, red);
    if (threadIdx.x == 0) {
        part[(size_t)l * nb + blockIdx.x] = num;
        part[(size_t)(L + l) * nb + blockIdx.x] = den;
    }
}

// lmax[l] = num / den from the k_trace_part partials (0 when den = 0).  grid L.
__global__ void k_trace_final(int L, const double* __restrict__ part, int nb, double* __restrict__ lmax) {
    __shared__ double red[16];
    const int l = blockIdx.x;
    const double a = sum_partials(part + (size_t)l * nb, nb, red);
    const double b = sum_partials(part + (size_t)(L + l) * nb, nb, red);
    if (threadIdx.x == 0) lmax[l] = b > 0.0 ? a / b : 0.0;
}
