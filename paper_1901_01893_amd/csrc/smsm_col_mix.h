// Normal-operator column pass for folded lengths with an odd factor
// (M = P Q, Q = 3 or 7, P a power of two: 24, 28, 48, 56 at n2 = 192, 224),
// with the contract of k_col<COL_NORMAL> (hybrid in -> hybrid out, the
// circular Hankel term from the tap table Kc).  The column image and the
// final ky transform are block-wide, as in k_col; the coil loop is
// register-resident, as in k_col_fast: wave w takes shot i = w % NS and the
// coils of coil group w / NS, lane l = grp M + m coil group member grp and
// folded point m (G = 64 / M members side by side, the remaining lanes idle).
// Per coil: fold, M-point DFT, CAIPI sum and split, inverse DFT, unfold into
// the lane's accumulators.  The M-point transforms run through a buffer of
// the wave's own in shared memory (no block barrier), as a two-factor
// decomposition (see wave_dft).
#pragma once
#include "smsm_kernels.h"

// Shared memory (double2 units): U [B][n2], ACC [B][n2], ky twiddles [n2],
// folded twiddles [M], the waves' transform buffers [NS CG][G][L][M], the
// regulariser's taps [L][Ns][Ns][nc], 16 for reductions.
__host__ __device__ inline int colmix_wb(int M, int L, int NS, int CG) { return NS * CG * (64 / M) * L * M; }
__host__ __device__ inline int colmix_lds_total(const Geo& g, int wb) {
    return 2 * g.B * g.n2 + g.n2 + g.M + wb + g.L * g.Ns * g.Ns * g.nc + 16;
}

SMSM_DEV void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Unnormalised DFT of length M = P Q (forward e^{-2 pi i jk/M}, INV e^{+...})
// of NV sequences held one point per lane (lane m holds point m of each),
// through the wave's buffer buf [NV][M] (this coil group's part):
//   X[k1 + P k2] = sum_{n2<Q} w^{P n2 k2} w^{n2 k1} sum_{n1<P} x[Q n1 + n2] w^{Q n1 k1}
// (n Q-major in, k P-minor out; w^{nk} splits because w^{M n1 k2} = 1).  Lane
// m forms the inner sum for (n2, k1) = (m / P, m % P) and stores it at m,
// then the outer for (k1, k2) = (m % P, m / P): output X[m], natural order.
// The powers of each sum's base are formed by repeated products from the
// table twm[k] = e^{-2 pi i k / M}.  Inactive lanes read but never write.
template <int M, int Q, int NV, bool INV>
SMSM_DEV void wave_dft(double2 (&f)[NV], double2* buf, const double2* twm, int m, bool active) {
    constexpr int P = M / Q;
    static_assert(P * Q == M && (P & (P - 1)) == 0, "M = P Q with P a power of two");
    auto tw = [&](int k) {
        const double2 w = twm[k];
        return INV ? cconj(w) : w;
    };
    if (active) {
#pragma unroll
        for (int v = 0; v < NV; ++v) buf[v * M + m] = f[v];
    }
    wave_fence();
    const int a = m / P, k1 = m % P;   // inner: n2 = a; outer: k2 = a
    double2 z[NV];
    {
        const double2 base = tw((Q * k1) % M), tz = tw((a * k1) % M);
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = cmk(0.0, 0.0);
        double2 wc = cmk(1.0, 0.0);   // w^{Q n1 k1}, shared by the NV sequences
#pragma unroll 4
        for (int n1 = 0; n1 < P; ++n1) {
#pragma unroll
            for (int v = 0; v < NV; ++v) z[v] = cfma(buf[v * M + Q * n1 + a], wc, z[v]);
            wc = cmul(wc, base);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) z[v] = cmul(z[v], tz);
    }
    wave_fence();
    if (active) {
#pragma unroll
        for (int v = 0; v < NV; ++v) buf[v * M + m] = z[v];
    }
    wave_fence();
    {
        const double2 base = tw((P * a) % M);
#pragma unroll
        for (int v = 0; v < NV; ++v) f[v] = cmk(0.0, 0.0);
        double2 wc = cmk(1.0, 0.0);   // w^{P n2 k2}
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) {
#pragma unroll
            for (int v = 0; v < NV; ++v) f[v] = cfma(buf[v * M + n2 * P + k1], wc, f[v]);
            wc = cmul(wc, base);
        }
    }
    wave_fence();
}

// grid (n1), block 64 NS CG (= 512).  n2 = M NS.
template <int M, int L, int NS, int CG>
__global__ void __launch_bounds__(64 * NS * CG)
k_col_mix(Geo g, const double2* __restrict__ h1, double2* __restrict__ h2, const double2* __restrict__ ST,
          const double2* __restrict__ theta, const double2* __restrict__ tau, const double2* __restrict__ tw2,
          const double2* __restrict__ twM, const double2* __restrict__ tw1, const double2* __restrict__ Kc,
          int use_reg) {
    constexpr int Q = (M % 7 == 0) ? 7 : 3;
    constexpr int G = 64 / M, B = L * NS, NW = NS * CG, N2 = M * NS;
    extern __shared__ double2 sm[];
    const int n1 = g.n1, Nc = g.Nc, nc = g.nc, e = g.e;
    const int x1 = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int i = wave % NS, cg = wave / NS;
    const int grp0 = lane / M, m = lane % M;
    const bool active = grp0 < G;
    const int grp = active ? grp0 : G - 1;
    double2* U = sm;
    double2* ACC = sm + B * N2;
    double2* TW2 = sm + 2 * B * N2;
    double2* TWM = TW2 + N2;
    double2* WB = TWM + M;
    double2* A = WB + colmix_wb(M, L, NS, CG);
    const double isq2 = 1.0 / sqrt((double)N2);
    const FastDiv dn2(N2);

    for (int k = tid; k < N2; k += nt) TW2[k] = tw2[k];
    for (int k = tid; k < M; k += nt) TWM[k] = twM[k];
    // image column u = centred inverse DFT along ky; stored as tau_i * u
    for (int idx = tid; idx < B * N2; idx += nt) {
        const int b = dn2.div(idx), j = idx - b * N2;
        U[idx] = cscale(h1[((size_t)b * n1 + x1) * N2 + j], sgn_pow(j));
    }
    fft_batch_lds(U, N2, g.logn2, B, N2, TW2, true);
    for (int idx = tid; idx < B * N2; idx += nt) {
        const int b = dn2.div(idx), n = idx - b * N2, ib = b % NS;
        U[idx] = cmul(tau[ib * N2 + n], cscale(U[idx], isq2 * sgn_pow(n)));
    }
    __syncthreads();

    // ---- coil loop: lane accumulators of positions n = m + M t, t < NS
    double2 acc[L][NS];
#pragma unroll
    for (int s = 0; s < L; ++s)
#pragma unroll
        for (int t = 0; t < NS; ++t) acc[s][t] = cmk(0.0, 0.0);
    const double2* Ui = U + i * N2 + m;
    double2 th[L];   // CAIPI phase of this lane's bin m (natural order)
#pragma unroll
    for (int s = 0; s < L; ++s) th[s] = theta[s * N2 + i + NS * m];
    double2* buf = WB + (wave * G + grp) * L * M;
    const int per_iter = CG * G;
    const int iters = (Nc + per_iter - 1) / per_iter;
    const size_t lane_off = (size_t)x1 * N2 + m;
    const size_t slice_stride = (size_t)Nc * n1 * N2, coil_stride = (size_t)n1 * N2;
#pragma unroll 1
    for (int it = 0; it < iters; ++it) {
        const int c = (it * CG + cg) * G + grp0;
        const double live = (active && c < Nc) ? 1.0 : 0.0;
        const size_t cbase = lane_off + (size_t)min(c, Nc - 1) * coil_stride;
        double2 sc[L][NS];
#pragma unroll
        for (int s = 0; s < L; ++s)
#pragma unroll
            for (int t = 0; t < NS; ++t) sc[s][t] = ST[cbase + s * slice_stride + M * t];
        double2 f[L];
#pragma unroll
        for (int s = 0; s < L; ++s) {
            double2 a = cmk(0.0, 0.0);
#pragma unroll
            for (int t = 0; t < NS; ++t) a = cfma(sc[s][t], Ui[s * NS * N2 + M * t], a);
            f[s] = cscale(a, live);
        }
        wave_dft<M, Q, L, false>(f, buf, TWM, m, active);
        double2 z = cmk(0.0, 0.0);
#pragma unroll
        for (int s = 0; s < L; ++s) z = cfma(th[s], f[s], z);
#pragma unroll
        for (int s = 0; s < L; ++s) f[s] = cmulc(z, th[s]);
        wave_dft<M, Q, L, true>(f, buf, TWM, m, active);
#pragma unroll
        for (int s = 0; s < L; ++s)
#pragma unroll
            for (int t = 0; t < NS; ++t) acc[s][t] = cadd(acc[s][t], cconjmul(sc[s][t], f[s]));
    }

    // ---- coil-group members of a wave: member g > 0 hands its sums to member 0
    // through the wave's buffer, in member order, one position t at a time
    if constexpr (G > 1) {
        double2* b0 = WB + wave * G * L * M;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
#pragma unroll
            for (int gg = 1; gg < G; ++gg) {
                if (grp0 == gg) {
#pragma unroll
                    for (int s = 0; s < L; ++s) b0[s * M + m] = acc[s][t];
                }
                wave_fence();
                if (grp0 == 0) {
#pragma unroll
                    for (int s = 0; s < L; ++s) acc[s][t] = cadd(acc[s][t], b0[s * M + m]);
                }
                wave_fence();
            }
        }
    }
    // ---- the coil groups of a shot through ACC, in order
    for (int k = 0; k < CG; ++k) {
        if (cg == k && grp0 == 0) {
#pragma unroll
            for (int s = 0; s < L; ++s)
#pragma unroll
                for (int t = 0; t < NS; ++t) {
                    const int o = (s * NS + i) * N2 + m + M * t;
                    ACC[o] = (k == 0) ? acc[s][t] : cadd(ACC[o], acc[s][t]);
                }
        }
        __syncthreads();
    }
    // normal-operator scaling conj(tau_i[n]) / n2
    for (int idx = tid; idx < B * N2; idx += nt) {
        const int b = dn2.div(idx), n = idx - b * N2, ib = b % NS;
        ACC[idx] = cscale(cmulc(ACC[idx], tau[ib * N2 + n]), 1.0 / (double)N2);
    }

    if (use_reg) hankel_image_term(g, x1, U, tw1, TW2, Kc, A, ACC, dn2, FastDiv(NS));
    __syncthreads();
    // centred forward DFT along ky
    for (int idx = tid; idx < B * N2; idx += nt) {
        const int n = idx - dn2.div(idx) * N2;
        ACC[idx] = cscale(ACC[idx], sgn_pow(n));
    }
    fft_batch_lds(ACC, N2, g.logn2, B, N2, TW2, false);
    for (int idx = tid; idx < B * N2; idx += nt) {
        const int b = dn2.div(idx), j = idx - b * N2;
        h2[((size_t)b * n1 + x1) * N2 + j] = cscale(ACC[idx], isq2 * sgn_pow(j));
    }
}
