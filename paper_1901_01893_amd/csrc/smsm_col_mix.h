// Normal-operator column pass for folded lengths with an odd factor
// (M = P Q, Q = 3 or 7, P a power of two: 24, 28, 48, 56, 96, 112 at
// n2 = 192, 224), with the contract of k_col<COL_NORMAL> (hybrid in -> hybrid
// out, the circular Hankel term from the per-column tap table of
// k_colmix_taps).  The column image and the final ky transform run in-wave
// by rows (ky_row_dft), the image-domain
// Hankel term runs over Hermitian shot pairs (hankel_image_pairs), and with
// pc.mode != 0 the pass also takes the
// CG direction update and the Re <p, Np> partial of its column, as
// k_col_fast does.  The coil loop is
// register-resident, as in k_col_fast: wave w takes shot i = w % NS and the
// coils of coil group w / NS.  M <= 64: lane l = grp M + a P + j is coil group
// member grp (G = 64 / M members side by side, the remaining lanes idle),
// group a < Q and place j < P, and holds folded point Q j + a.  M > 64: one
// member, two points per lane: lane a' P + j holds groups a = a' + (64 / P) r
// in its registers r = 0, 1 (the slots with a >= Q idle).
// Per coil: fold, M-point DFT, CAIPI sum and split, inverse DFT, unfold into
// the lane's accumulators (see mix_dft for the transforms).
#pragma once
#include "smsm_col_fast.h"

// Shared memory (double2 units): U [B][n2], ACC [B][n2], ky twiddles [n2],
// folded twiddles [M], the waves' transform buffers [NS CG][G][L][M], the
// regulariser's taps [L][Ns][Ns][nc], 16 for reductions.
__host__ __device__ inline int colmix_wb(int M, int L, int NS, int CG) {
    return NS * CG * (M > 64 ? 1 : 64 / M) * L * M;
}
__host__ __device__ inline int colmix_lds_total(const Geo& g, int wb) {
    return 2 * g.B * g.n2 + g.n2 + g.M + wb + g.L * g.Ns * g.Ns * g.nc + 16;
}

SMSM_DEV void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-lane constants of the M = P Q point transforms (twm[k] = e^{-2 pi i k/M}):
// the radix-2 stage twiddles and signs of the P-point transform across the P
// lanes of a group, and per register r the inter-factor twiddle
// w_M^(a_r brev(j)) and the base w_Q^(a_r) of the Q-point sums.  Built from
// the shared-memory table at each transform (a few independent reads), so
// they hold no registers across the coil loop.
template <int M, int Q, int MR>
struct MixLane {
    static constexpr int P = M / Q;
    static constexpr int LOGP = P == 32 ? 5 : P == 16 ? 4 : P == 8 ? 3 : 2;
    static_assert(P * Q == M && (P == 4 || P == 8 || P == 16 || P == 32), "M = P Q with P = 4 .. 32");
    double2 w[8];
    double sg[8];
    double2 tf[MR], tq[MR];
    SMSM_DEV void setup(const double2* twm, int j, const int (&a)[MR]) {
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int h = 1 << st;
            const bool upper = (j & h) == 0;
            sg[st] = upper ? 1.0 : -1.0;
            w[st] = (st >= LOGP || upper) ? cmk(1.0, 0.0) : twm[(j & (h - 1)) * (M / (2 * h))];
        }
        const int bj = (int)(__brev((unsigned)j) >> (32 - LOGP));
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            tf[r] = twm[a[r] * bj];
            tq[r] = twm[P * a[r]];
        }
    }
};

// Q-point sums through the wave's buffer buf [L][M] (this member's part):
// slot (a, j) stores its value at a P + j, then forms
//   sum_{a' < Q} buf[a' P + j] (w_Q^{+-a})^{a'}
// (the powers of the base by repeated products).  Idle slots read but never
// write.
template <int M, int Q, int L, int MR, bool INV>
SMSM_DEV void mix_qsum(double2 (&f)[L * MR], double2* buf, const MixLane<M, Q, MR>& c, int j,
                       const int (&a)[MR], const bool (&ok)[MR]) {
    constexpr int P = M / Q;
#pragma unroll
    for (int r = 0; r < MR; ++r)
        if (ok[r]) {
#pragma unroll
            for (int s = 0; s < L; ++s) buf[s * M + a[r] * P + j] = f[s * MR + r];
        }
    wave_fence();
    double2 base[MR], wc[MR];
#pragma unroll
    for (int r = 0; r < MR; ++r) {
        base[r] = INV ? cconj(c.tq[r]) : c.tq[r];
        wc[r] = cmk(1.0, 0.0);
    }
#pragma unroll
    for (int v = 0; v < L * MR; ++v) f[v] = cmk(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const double2 x = buf[s * M + q * P + j];
#pragma unroll
            for (int r = 0; r < MR; ++r) f[s * MR + r] = cfma(x, wc[r], f[s * MR + r]);
        }
#pragma unroll
        for (int r = 0; r < MR; ++r) wc[r] = cmul(wc[r], base[r]);
    }
    wave_fence();
}

// Unnormalised M-point DFT (forward e^{-2 pi i nk/M}, INV e^{+...}) of L
// sequences (MR slots each), M = P Q, n = Q n1 + a, k = k1 + P k2:
//   X[k1 + P k2] = sum_a w_Q^(a k2) w_M^(a k1) sum_{n1 < P} x[Q n1 + a] w_P^(n1 k1)
// (w_M^(nk) splits because w_M^(Q n1 P k2) = 1).  Forward: slot (a, j) holds
// x[Q j + a]; the P-point transform runs across the lanes of group a
// (decimation in frequency, leaving k1 = brev(j)), then the twiddle, then the
// Q-point sum of mix_qsum leaves X[brev(j) + P a] in slot (a, j).  The inverse
// is the conjugate transpose: Q-point sums, conjugate twiddle, decimation in
// time across the group (bit-reversed in, natural out), back to the slot's
// point Q j + a.
template <int M, int Q, int L, int MR, bool INV>
SMSM_DEV void mix_dft(double2 (&f)[L * MR], double2* buf, const double2* twm, int j, const int (&a)[MR],
                      const bool (&ok)[MR]) {
    constexpr int P = M / Q;
    MixLane<M, Q, MR> c;
    c.setup(twm, j, a);
    if constexpr (!INV) {
        fft_dif<P, L * MR>(f, c.w, c.sg);
#pragma unroll
        for (int s = 0; s < L; ++s)
#pragma unroll
            for (int r = 0; r < MR; ++r) f[s * MR + r] = cmul(f[s * MR + r], c.tf[r]);
        mix_qsum<M, Q, L, MR, false>(f, buf, c, j, a, ok);
    } else {
        mix_qsum<M, Q, L, MR, true>(f, buf, c, j, a, ok);
#pragma unroll
        for (int s = 0; s < L; ++s)
#pragma unroll
            for (int r = 0; r < MR; ++r) f[s * MR + r] = cmulc(f[s * MR + r], c.tf[r]);
        fft_dit_inv<P, L * MR>(f, c.w, c.sg);
    }
}

// In-wave ky DFT of rows of length N2 = RQ RL (RQ = 3 or 7, RL = 16, 32 or 64
// lanes per row, 64 / RL rows per wave): lane j of a row holds x[j + RL t],
// t < RQ.  With n = j + RL t and k = k1 + RQ k2,
//   X[k1 + RQ k2] = sum_j w_RL^(j k2) w_N2^(j k1) sum_t x[j + RL t] w_RQ^(t k1),
// so the RQ-point DFT of the lane's own values, the twiddle w_N2^(j k1) and
// the RL-point transform across the row's lanes (decimation in frequency)
// leave X[k1 + RQ brev(j)] in register k1 (unnormalised; INV: the conjugate
// transform).  TW2[k] = e^{-2 pi i k / N2} (shared memory).
template <int N2>
struct KyRow {
    static constexpr int RQ = N2 % 7 == 0 ? 7 : 3, RL = N2 / RQ;
    static constexpr int LOGL = RL == 64 ? 6 : RL == 32 ? 5 : RL == 16 ? 4 : 3;
    static_assert(RQ * RL == N2 && (RL & (RL - 1)) == 0 && RL >= 8 && RL <= 64, "n2 = RQ 2^a, 8 <= 2^a <= 64");
};

template <bool INV>
SMSM_DEV double2 tw_at(const double2* TW2, int k) {
    const double2 w = TW2[k];
    return INV ? cconj(w) : w;
}

template <int N2, bool INV>
SMSM_DEV void ky_row_dft(double2 (&x)[KyRow<N2>::RQ], const double2* TW2, int j) {
    constexpr int RQ = KyRow<N2>::RQ, RL = KyRow<N2>::RL, LOGL = KyRow<N2>::LOGL;
    double2 y[RQ];
#pragma unroll
    for (int k1 = 0; k1 < RQ; ++k1) {
        double2 sum = x[0];
#pragma unroll
        for (int t = 1; t < RQ; ++t) sum = cfma(x[t], tw_at<INV>(TW2, ((t * k1) % RQ) * RL), sum);
        y[k1] = k1 == 0 ? sum : cmul(sum, tw_at<INV>(TW2, j * k1));
    }
    double2 w[8];
    double sg[8];
#pragma unroll
    for (int st = 0; st < 8; ++st) {
        const int h = 1 << st;
        const bool upper = (j & h) == 0;
        sg[st] = upper ? 1.0 : -1.0;
        w[st] = (st >= LOGL || upper) ? cmk(1.0, 0.0) : tw_at<INV>(TW2, (j & (h - 1)) * (N2 / (2 * h)));
    }
    fft_dif<RL, RQ>(y, w, sg);
#pragma unroll
    for (int k1 = 0; k1 < RQ; ++k1) x[k1] = y[k1];
}

// Per-column tap table of the image-domain Hankel term, built once per weight
// update (grid n1): At[x1][l][i][j][d2] = sum_d1 Kc[l][i][j][d2][d1] w1^(d1 - e),
// w1 = e^{-2 pi i (x1 - n1/2)/n1}, by Horner's rule in w1 (the arithmetic of
// hankel_image_term's table), so that the column pass copies its column's
// L Ns Ns nc entries instead of every workgroup re-reading all of Kc.
__global__ void __launch_bounds__(256) k_colmix_taps(Geo g, const double2* __restrict__ Kc,
                                                     const double2* __restrict__ tw1, double2* __restrict__ At) {
    const int x1 = blockIdx.x, n1 = g.n1, nc = g.nc, e = g.e;
    const int ntap = g.L * g.Ns * g.Ns * nc;
    const int nu1 = x1 - n1 / 2;
    const double2 w1 = tw1[imod(nu1, n1)], w1e = tw1[imod(-e * nu1, n1)];
    for (int idx = threadIdx.x; idx < ntap; idx += blockDim.x) {
        const double2* kr = Kc + (size_t)idx * nc;
        double2 kv[BAND_MAX_NC];
#pragma unroll
        for (int d1 = 0; d1 < BAND_MAX_NC; ++d1)
            if (d1 < nc) kv[d1] = kr[d1];
        double2 p = cmk(0.0, 0.0);
#pragma unroll
        for (int d1 = BAND_MAX_NC - 1; d1 >= 0; --d1)
            if (d1 < nc) p = cfma(p, w1, kv[d1]);
        At[(size_t)x1 * ntap + idx] = cmul(p, w1e);
    }
}

// Image-domain Hankel term (that of hankel_image_term) by points, each shot pair
// once: W is Hermitian, so Kc[l][i][j][d] = conj(Kc[l][j][i][2e - d]) and the
// evaluated kernel K[l][i][j](x, n) = conj(K[l][j][i](x, n)).  A thread takes
// a point (l, n), evaluates K[l][i][j] for i <= j by Horner's rule and adds
// K u_i to output shot j and conj(K) u_j to output shot i: NS (NS + 1) / 2
// tap sums per point instead of NS^2.  The column's taps come from the table
// of k_colmix_taps (At).
template <int NS>
SMSM_DEV void hankel_image_pairs(const Geo& g, int x1, const double2* U, const double2* __restrict__ At,
                                 const double2* TW2, double2* A, double2* ACC, const FastDiv& dn2) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n2 = g.n2, nc = g.nc, e = g.e;
    const int ntap = g.L * NS * NS * nc;
    const double2* Ac = At + (size_t)x1 * ntap;
    for (int idx = tid; idx < ntap; idx += nt) A[idx] = Ac[idx];
    __syncthreads();
    for (int item = tid; item < g.L * n2; item += nt) {
        const int l = dn2.div(item), n = item - l * n2;
        const double2 w2 = TW2[imod(n - n2 / 2, n2)], w2e = TW2[imod(-e * (n - n2 / 2), n2)];
        double2 u[NS], acc[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int k = i * n - n2 * dn2.div(i * n);
            u[i] = cmulc(U[(l * NS + i) * n2 + n], cscale(TW2[k], sgn_pow(n)));
            acc[i] = cmk(0.0, 0.0);
        }
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int j = i; j < NS; ++j) {
                const double2* ar = A + (size_t)((l * NS + i) * NS + j) * nc;
                double2 p = cmk(0.0, 0.0);
                for (int d2 = nc - 1; d2 >= 0; --d2) p = cfma(p, w2, ar[d2]);
                const double2 kij = cmul(p, w2e);
                acc[j] = cfma(kij, u[i], acc[j]);
                if (j != i) acc[i] = cfma(cconj(kij), u[j], acc[i]);
            }
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int o = (l * NS + j) * n2 + n;
            ACC[o] = cadd(ACC[o], acc[j]);
        }
    }
}

// grid (n1), block 64 NS CG (= 512).  n2 = M NS.  With pc.mode != 0 the pass
// also takes the CG direction update of its column (p = r, or x += alpha p_old
// and p = r + beta p_old with beta from the |r|^2 partials) as it loads the
// rows, and writes its column's Re <p, output> partial to pc.pq[blockIdx.x],
// formed in the image domain (the ky transforms are unitary).
template <int M, int L, int NS, int CG>
__global__ void __launch_bounds__(64 * NS * CG)
k_col_mix(Geo g, const double2* __restrict__ h1, double2* __restrict__ h2, const double2* __restrict__ ST,
          const double2* __restrict__ theta, const double2* __restrict__ tau, const double2* __restrict__ tw2,
          const double2* __restrict__ twM, const double2* __restrict__ At, int use_reg, ColCg pc) {
    constexpr int Q = (M % 7 == 0) ? 7 : 3, P = M / Q;
    constexpr int MR = M > 64 ? 2 : 1;          // folded points per lane
    constexpr int G = M > 64 ? 1 : 64 / M;      // coil-group members per wave
    constexpr int GL = 64 / P;                  // lane groups per register (MR = 2)
    constexpr int B = L * NS, NW = NS * CG, N2 = M * NS;
    static_assert(MR == 1 || Q <= 2 * GL, "two slots per lane cover the Q groups");
    extern __shared__ double2 sm[];
    const int n1 = g.n1, Nc = g.Nc, nc = g.nc, e = g.e;
    const int x1 = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int i = wave % NS, cg = wave / NS;
    const int grp0 = MR == 1 ? lane / M : 0;
    const int m = MR == 1 ? lane % M : lane;   // lane within its member
    const int j = m % P;
    const bool active = grp0 < G;
    const int grp = active ? grp0 : G - 1;
    int a[MR], tpos[MR];   // each slot's group and folded point
    bool ok[MR];
#pragma unroll
    for (int r = 0; r < MR; ++r) {
        const int ar = m / P + GL * r;
        ok[r] = active && ar < Q;
        a[r] = min(ar, Q - 1);
        tpos[r] = Q * j + a[r];
    }
    double2* U = sm;
    double2* ACC = sm + B * N2;
    double2* TW2 = sm + 2 * B * N2;
    double2* TWM = TW2 + N2;
    double2* WB = TWM + M;
    double2* A = WB + colmix_wb(M, L, NS, CG);
    const double isq2 = 1.0 / sqrt((double)N2);
    const FastDiv dn2(N2);

    double* red = (double*)(sm + colmix_lds_total(g, colmix_wb(M, L, NS, CG)) - 16);
    for (int k = tid; k < N2; k += nt) TW2[k] = tw2[k];
    for (int k = tid; k < M; k += nt) TWM[k] = twM[k];
    double beta = 0.0;
    const double alpha_prev = (pc.mode == 2 && pc.x) ? *pc.alpha_prev : 0.0;
    if (pc.mode != 0) {
        const double rn = sum_partials(pc.rr_new, pc.nrr, red);
        if (pc.mode == 2) {
            const double ro = *pc.rr_old;
            beta = ro > 0.0 ? rn / ro : 0.0;
        }
        if (x1 == 0 && tid == 0) *pc.rr_out = rn;
    }
    __syncthreads();
    // ky rows in-wave: wave w takes rows w RG + lane / RL, + NW RG per step
    constexpr int RQ = KyRow<N2>::RQ, RL = KyRow<N2>::RL, RG = 64 / RL;
    // image column u = centred inverse DFT along ky; stored as tau_i * u,
    // tau_i[n] = (-1)^n w_n2^(i n) (bitwise the host table)
    for (int b0 = wave * RG; b0 < B; b0 += NW * RG) {
        const int b = b0 + lane / RL, bc = min(b, B - 1), jr = lane % RL;
        double2 x[RQ];
#pragma unroll
        for (int t = 0; t < RQ; ++t) {
            const int n = jr + RL * t;
            const size_t k0 = ((size_t)bc * n1 + x1) * N2 + n;
            double2 val;
            if (pc.mode == 0) {
                val = h1[k0];
            } else {
                // rows past B (clamped) read only; their results are dropped
                val = pc.r[k0];
                if (pc.mode == 2) {
                    const double2 po = pc.p_old[k0];
                    if (pc.x && b < B) pc.x[k0] = cadd(pc.x[k0], cscale(po, alpha_prev));
                    val = cadd(val, cscale(po, beta));
                }
                if (b < B) pc.p[k0] = val;
            }
            x[t] = cscale(val, sgn_pow(n));
        }
        ky_row_dft<N2, true>(x, TW2, jr);
        if (b < B) {
            const int ib = b % NS, bjr = (int)(__brev((unsigned)jr) >> (32 - KyRow<N2>::LOGL));
#pragma unroll
            for (int k1 = 0; k1 < RQ; ++k1) {
                const int n = k1 + RQ * bjr, k = ib * n - N2 * dn2.div(ib * n);
                U[b * N2 + n] = cmul(cscale(TW2[k], sgn_pow(n)), cscale(x[k1], isq2 * sgn_pow(n)));
            }
        }
    }
    __syncthreads();

    // ---- coil loop: slot accumulators of positions n = tpos + M t, t < NS
    double2 acc[L][NS][MR];
#pragma unroll
    for (int s = 0; s < L; ++s)
#pragma unroll
        for (int t = 0; t < NS; ++t)
#pragma unroll
            for (int r = 0; r < MR; ++r) acc[s][t][r] = cmk(0.0, 0.0);
    const double2* Ui = U + i * N2;
    // CAIPI phase of each slot's bin after the forward transform
    const int bj = (int)(__brev((unsigned)j) >> (32 - MixLane<M, Q, MR>::LOGP));
    double2 th[L][MR];
#pragma unroll
    for (int s = 0; s < L; ++s)
#pragma unroll
        for (int r = 0; r < MR; ++r) th[s][r] = theta[s * N2 + i + NS * (bj + P * a[r])];
    double2* buf = WB + (wave * G + grp) * L * M;
    const int per_iter = CG * G;
    const int iters = (Nc + per_iter - 1) / per_iter;
    const size_t col_off = (size_t)x1 * N2;
    const size_t slice_stride = (size_t)Nc * n1 * N2, coil_stride = (size_t)n1 * N2;
#pragma unroll 1
    for (int it = 0; it < iters; ++it) {
        const int c = (it * CG + cg) * G + grp0;
        const size_t cbase = col_off + (size_t)min(c, Nc - 1) * coil_stride;
        double2 sc[L][NS][MR];
#pragma unroll
        for (int s = 0; s < L; ++s)
#pragma unroll
            for (int t = 0; t < NS; ++t)
#pragma unroll
                for (int r = 0; r < MR; ++r) sc[s][t][r] = ST[cbase + s * slice_stride + tpos[r] + M * t];
        double2 f[L * MR];
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            const double live = (ok[r] && c < Nc) ? 1.0 : 0.0;
#pragma unroll
            for (int s = 0; s < L; ++s) {
                double2 v = cmk(0.0, 0.0);
#pragma unroll
                for (int t = 0; t < NS; ++t) v = cfma(sc[s][t][r], Ui[s * NS * N2 + tpos[r] + M * t], v);
                f[s * MR + r] = cscale(v, live);
            }
        }
        mix_dft<M, Q, L, MR, false>(f, buf, TWM, j, a, ok);
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            double2 z = cmk(0.0, 0.0);
#pragma unroll
            for (int s = 0; s < L; ++s) z = cfma(th[s][r], f[s * MR + r], z);
#pragma unroll
            for (int s = 0; s < L; ++s) f[s * MR + r] = cmulc(z, th[s][r]);
        }
        mix_dft<M, Q, L, MR, true>(f, buf, TWM, j, a, ok);
#pragma unroll
        for (int s = 0; s < L; ++s)
#pragma unroll
            for (int t = 0; t < NS; ++t)
#pragma unroll
                for (int r = 0; r < MR; ++r)
                    acc[s][t][r] = cadd(acc[s][t][r], cconjmul(sc[s][t][r], f[s * MR + r]));
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
                    for (int s = 0; s < L; ++s) b0[s * M + m] = acc[s][t][0];
                }
                wave_fence();
                if (grp0 == 0) {
#pragma unroll
                    for (int s = 0; s < L; ++s) acc[s][t][0] = cadd(acc[s][t][0], b0[s * M + m]);
                }
                wave_fence();
            }
        }
    }
    // ---- the coil groups of a shot through ACC, in order
    for (int k = 0; k < CG; ++k) {
        if (cg == k && grp0 == 0) {
#pragma unroll
            for (int r = 0; r < MR; ++r)
                if (ok[r]) {
#pragma unroll
                    for (int s = 0; s < L; ++s)
#pragma unroll
                        for (int t = 0; t < NS; ++t) {
                            const int o = (s * NS + i) * N2 + tpos[r] + M * t;
                            ACC[o] = (k == 0) ? acc[s][t][r] : cadd(ACC[o], acc[s][t][r]);
                        }
                }
        }
        __syncthreads();
    }
    // normal-operator scaling conj(tau_i[n]) / n2
    for (int idx = tid; idx < B * N2; idx += nt) {
        const int b = dn2.div(idx), n = idx - b * N2, ib = b % NS;
        ACC[idx] = cscale(cmulc(ACC[idx], tau[ib * N2 + n]), 1.0 / (double)N2);
    }

    if (use_reg) hankel_image_pairs<NS>(g, x1, U, At, TW2, A, ACC, dn2);
    __syncthreads();
    // Re <p, output> = Re <u, ACC> with u = conj(tau) U (unitary ky transforms)
    if (pc.mode != 0) {
        double dot = 0.0;
        for (int idx = tid; idx < B * N2; idx += nt) {
            const int b = dn2.div(idx), n = idx - b * N2, ib = b % NS;
            const int k = ib * n - N2 * dn2.div(ib * n);
            const double2 cu = cmul(cscale(TW2[k], sgn_pow(n)), cconj(U[idx]));   // conj(u)
            const double2 a = ACC[idx];
            dot += cu.x * a.x - cu.y * a.y;
        }
        dot = block_sum(dot, red);
        if (tid == 0) pc.pq[blockIdx.x] = dot;
    }
    // centred forward DFT along ky, in-wave by rows; a wave reorders its own
    // rows through ACC for a coalesced store
    for (int b0 = wave * RG; b0 < B; b0 += NW * RG) {
        const int b = b0 + lane / RL, bc = min(b, B - 1), jr = lane % RL;
        double2 x[RQ];
#pragma unroll
        for (int t = 0; t < RQ; ++t) {
            const int n = jr + RL * t;
            x[t] = cscale(ACC[bc * N2 + n], sgn_pow(n));
        }
        ky_row_dft<N2, false>(x, TW2, jr);
        wave_fence();
        if (b < B) {
            const int bjr = (int)(__brev((unsigned)jr) >> (32 - KyRow<N2>::LOGL));
#pragma unroll
            for (int k1 = 0; k1 < RQ; ++k1) {
                const int n = k1 + RQ * bjr;
                ACC[b * N2 + n] = cscale(x[k1], isq2 * sgn_pow(n));
            }
        }
        wave_fence();
        if (b < B) {
#pragma unroll
            for (int t = 0; t < RQ; ++t) {
                const int n = jr + RL * t;
                h2[((size_t)b * n1 + x1) * N2 + n] = ACC[b * N2 + n];
            }
        }
    }
}
