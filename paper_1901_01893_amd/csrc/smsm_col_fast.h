// Register-resident column kernel for the SENSE coil loop of the normal
// operator (one workgroup per image column x).
//
// Wave w handles shot i = w % NS and the coils of coil group w / NS.  Inside a
// wave, lane l = g*M + m works on coil group member g and folded ky point m;
// it keeps the coil-summed accumulator of every slice s and fold index t in
// registers and reads tau_i * u_{s,i}[m + M t] from shared memory.  Per coil:
//   fold     f_s[m]  = sum_t S_{s,c}[m + M t] (tau_i u_{s,i})[m + M t]
//   forward  M-point DFT across the M lanes of the group (decimation in
//            frequency: natural order in, bit-reversed order out)
//   CAIPI    Z = sum_s theta_s Y_s ;  Y'_s = conj(theta_s) Z   (pointwise)
//   inverse  M-point inverse DFT (decimation in time: bit-reversed in,
//            natural order out)
//   unfold   acc_s[t] += conj(S_{s,c}[m + M t]) g_s[m]
// Lane exchanges use DPP for xor distances 1, 2 and 8 and the LDS crossbar
// (ds_swizzle / ds_bpermute) for 4, 16 and 32; all 64 lanes stay active
// through every exchange.
#pragma once
#include "smsm_kernels.h"

template <int CTRL>
SMSM_DEV double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// xor 4, xor 16 and xor 32 go through the LDS crossbar (ds_swizzle in xor
// mode within 32-lane halves, ds_bpermute across halves): they issue on the
// LDS pipe and leave the vector ALU to the butterflies.  (A DPP pair or a
// permlane swap plus select costs two VALU issues per dword; xor 1, 2 and 8
// are single DPP moves and stay on the vector ALU, which measured faster than
// moving them to the LDS pipe as well.)
template <int H>
SMSM_DEV double swz_xor_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffLL), 0x1F | (H << 10));
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x1F | (H << 10));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
SMSM_DEV double perm_xor32_d(double v) {
    const long long b = __double_as_longlong(v);
    const int addr = (int)(((threadIdx.x & 63) ^ 32) << 2);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// value of lane (l ^ MASK)
template <int MASK>
SMSM_DEV double lane_xor(double v) {
    if constexpr (MASK == 1) return dpp_d<0xB1>(v);                 // quad_perm [1,0,3,2]
    else if constexpr (MASK == 2) return dpp_d<0x4E>(v);            // quad_perm [2,3,0,1]
    else if constexpr (MASK == 4) return swz_xor_d<4>(v);
    else if constexpr (MASK == 8) return dpp_d<0x128>(v);           // row_ror:8 (within 16 lanes: ^8)
    else if constexpr (MASK == 16) return swz_xor_d<16>(v);
    else return perm_xor32_d(v);
}

template <int MASK>
SMSM_DEV double2 lane_xor2(double2 v) {
    return make_double2(lane_xor<MASK>(v.x), lane_xor<MASK>(v.y));
}

// One decimation-in-frequency stage of span H on NV values:
// upper lane (bit H clear): a + b ; lower lane: (a - b) w.  At span 1 every
// twiddle is 1 and the multiply is skipped.
template <int H, int NV>
SMSM_DEV void dif_stage(double2 (&v)[NV], double sgn, double2 w) {
#pragma unroll
    for (int s = 0; s < NV; ++s) {
        const double2 p = lane_xor2<H>(v[s]);
        const double2 d = make_double2(p.x + sgn * v[s].x, p.y + sgn * v[s].y);
        v[s] = H == 1 ? d : cmul(d, w);
    }
}

// One decimation-in-time stage of span H with conjugated twiddle:
// upper: u + conj(w) v ; lower: u - conj(w) v (twiddle 1 at span 1).
template <int H, int NV>
SMSM_DEV void dit_stage(double2 (&v)[NV], double sgn, double2 w) {
    const double2 wc = cconj(w);
#pragma unroll
    for (int s = 0; s < NV; ++s) {
        const double2 t = H == 1 ? v[s] : cmul(wc, v[s]);   // upper lanes: w = 1, so t = own value
        const double2 p = lane_xor2<H>(t);
        v[s] = make_double2(p.x + sgn * t.x, p.y + sgn * t.y);
    }
}

template <int M, int NV>
SMSM_DEV void fft_dif(double2 (&v)[NV], const double2 (&w)[8], const double (&sg)[8]) {
    if constexpr (M >= 64) dif_stage<32, NV>(v, sg[5], w[5]);
    if constexpr (M >= 32) dif_stage<16, NV>(v, sg[4], w[4]);
    if constexpr (M >= 16) dif_stage<8, NV>(v, sg[3], w[3]);
    if constexpr (M >= 8) dif_stage<4, NV>(v, sg[2], w[2]);
    if constexpr (M >= 4) dif_stage<2, NV>(v, sg[1], w[1]);
    dif_stage<1, NV>(v, sg[0], w[0]);
}

template <int M, int NV>
SMSM_DEV void fft_dit_inv(double2 (&v)[NV], const double2 (&w)[8], const double (&sg)[8]) {
    dit_stage<1, NV>(v, sg[0], w[0]);
    if constexpr (M >= 4) dit_stage<2, NV>(v, sg[1], w[1]);
    if constexpr (M >= 8) dit_stage<4, NV>(v, sg[2], w[2]);
    if constexpr (M >= 16) dit_stage<8, NV>(v, sg[3], w[3]);
    if constexpr (M >= 32) dit_stage<16, NV>(v, sg[4], w[4]);
    if constexpr (M >= 64) dit_stage<32, NV>(v, sg[5], w[5]);
}

// Shared-memory layout (double2 units) of k_col_fast: U, ACC, ky twiddles.
__host__ __device__ inline int colfast_lds_total(const Geo& g) { return 2 * g.B * g.n2 + g.n2 + 16; }

// Image-domain kernel of the circular Hankel term, one table per IRLS step:
//   Khat[l][j][i][x][n] = sum_{d2,d1} Kc[l][j][i][d2][d1] e^{-2 pi i ((d1-e)(x-n1/2)/n1 + (d2-e)(n-n2/2)/n2)}
// (input shot j, output shot i).  W is Hermitian, so Kc[l][i][j][d] =
// conj(Kc[l][j][i][2e - d]) and Khat[l][i][j] = conj(Khat[l][j][i]): only the
// pairs j <= i are stored, pair p = i (i + 1) / 2 + j (khat_pair), as
// Khat[l][p][x][n].  grid (n1, L Ns (Ns + 1) / 2), block 256: the taps' x
// transform A[d2] (products formed in parallel, summed in d1 order), then one
// output n per thread from shared-memory twiddles.  f32: the table is written
// as complex64 (same element index, half the bytes), read back widened.
SMSM_HD inline int khat_pair(int j, int i) { return i * (i + 1) / 2 + j; }   // j <= i
__global__ void __launch_bounds__(256) k_hankel_image(Geo g, const double2* __restrict__ Kc,
                                                      const double2* __restrict__ tw1,
                                                      const double2* __restrict__ tw2, double2* __restrict__ Khat,
                                                      int f32) {
    __shared__ double2 A[BAND_MAX_NC];
    __shared__ double2 PR[BAND_MAX_NC * BAND_MAX_NC];
    __shared__ double2 T2[256];
    const int np = g.Ns * (g.Ns + 1) / 2, s = blockIdx.y / np, p = blockIdx.y - s * np;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= p) ++i;
    const int j = p - i * (i + 1) / 2;
    const int x = blockIdx.x, sji = (s * g.Ns + j) * g.Ns + i, nc = g.nc, e = g.e, n1 = g.n1, n2 = g.n2;
    const int nu1 = x - n1 / 2;
    for (int n = threadIdx.x; n < n2; n += blockDim.x) T2[n] = tw2[n];
    for (int t = threadIdx.x; t < nc * nc; t += blockDim.x) {
        const int d1 = t % nc;
        PR[t] = cmul(Kc[(size_t)sji * nc * nc + t], tw1[((d1 - e) * nu1) & (n1 - 1)]);
    }
    __syncthreads();
    if (threadIdx.x < nc) {
        double2 a = cmk(0.0, 0.0);
        for (int d1 = 0; d1 < nc; ++d1) a = cadd(a, PR[threadIdx.x * nc + d1]);
        A[threadIdx.x] = a;
    }
    __syncthreads();
    for (int n = threadIdx.x; n < n2; n += blockDim.x) {
        double2 k = cmk(0.0, 0.0);
        for (int d2 = 0; d2 < nc; ++d2) k = cfma(A[d2], T2[((d2 - e) * (n - n2 / 2)) & (n2 - 1)], k);
        const size_t o = ((size_t)blockIdx.y * n1 + x) * n2 + n;
        if (f32) reinterpret_cast<float2*>(Khat)[o] = make_float2((float)k.x, (float)k.y);   // complex64 form
        else Khat[o] = k;
    }
}

template <int N> struct WaveFft;

// Optional CG direction update fused into the column pass (hybrid layout):
// mode 0: the input is h1; mode 1: p = r; mode 2: p = r + beta p_old with
// beta = sum(rr_new[0..nrr)) / *rr_old (0 when *rr_old is 0), and, when x is
// given, the previous step x += (*alpha_prev) p_old on the way (the vector
// update of that step left x alone).
// In modes 1 and 2 the new p is written to p (p_old may be the same buffer:
// each element is read before it is written, by the same thread) and the
// input is p; each
// workgroup also stores Re <p, output> of its column in pq[blockIdx.x],
// evaluated in the image domain (the ky transforms are unitary), and the
// first workgroup stores sum(rr_new[0..nrr)) (the new |r|^2) in *rr_out for
// the step length of the vector update.
struct ColCg {
    const double2* r;
    const double2* p_old;    // the previous direction (mode 2)
    double2* p;
    double2* x;              // iterate that takes the previous step (mode 2), or null
    const double* alpha_prev;   // that step's length (scalar)
    const double* rr_new;    // partials of the new |r|^2
    int nrr;
    const double* rr_old;    // the previous |r|^2 (scalar)
    int mode;
    double* pq;
    double* rr_out;          // receives the new |r|^2 (scalar)
};

// Normal operator column pass; same input/output contract as k_col<COL_NORMAL>.
// Also writes prow[b][j][x] (the input's rows within 2e of the ky edges, j as
// in k_band_extract) for the band kernel.
// Template: M = n2/Ns (folded length, 8 to 128), L slices, NS shots, CG coil
// groups (waves per shot), KF32: Khat stored complex64 (the mixed-precision
// form).  blockDim.x = 64 * NS * CG.  n2 = M * NS >= 64.
template <int M, int L, int NS, int CG, bool KF32 = false>
__global__ void __launch_bounds__(64 * NS * CG)
k_col_fast(Geo g, const double2* __restrict__ h1, double2* __restrict__ h2, const double2* __restrict__ ST,
           const double2* __restrict__ theta, const double2* __restrict__ tw2, const double2* __restrict__ twM,
           const double2* __restrict__ Khat, int use_reg, ColCg pc, double2* __restrict__ prow) {
    constexpr int N2 = M * NS;
    // M <= 64: a folded sequence spans ML = M lanes (G = 64 / M coils side by
    // side); M = 128: each lane holds MR = 2 of its points (m and m + 64), the
    // first transform stage is in registers and the rest spans the 64 lanes.
    constexpr int MR = M > 64 ? M / 64 : 1, ML = M / MR;
    static_assert(MR == 1 || MR == 2, "folded lengths up to 128");
    constexpr int TQ = NS * MR;    // positions per lane: n = m + ML q, q < TQ
    constexpr int G = 64 / ML;     // coils processed side by side in one wave
    constexpr int LOGM = (ML == 8) ? 3 : (ML == 16) ? 4 : (ML == 32) ? 5 : 6;
    constexpr int B = L * NS, NW = NS * CG;
    using FC = WaveFft<N2>;
    constexpr int RC = FC::R;
    extern __shared__ double2 sm[];
    const int n1 = g.n1, Nc = g.Nc;
    const int x1 = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int i = wave % NS, cg = wave / NS;
    const int grp = lane / ML, m = lane % ML;
    double2* U = sm;
    double2* ACC = sm + B * N2;
    double2* TW2 = sm + 2 * B * N2;
    const double isq2 = 1.0 / sqrt((double)N2);

    for (int k = tid; k < N2; k += nt) TW2[k] = tw2[k];
    double beta = 0.0;
    const double alpha_prev = (pc.mode == 2 && pc.x) ? *pc.alpha_prev : 0.0;
    if (pc.mode != 0) {
        const double rn = sum_partials(pc.rr_new, pc.nrr, (double*)ACC);
        if (pc.mode == 2) {
            const double ro = *pc.rr_old;
            beta = ro > 0.0 ? rn / ro : 0.0;
        }
        if (x1 == 0 && tid == 0) *pc.rr_out = rn;
    }
    __syncthreads();

    // ---- column image: U[b][n] = tau_i[n] u_b[n], u_b = centred inverse DFT along ky of h1 column
    for (int b = wave; b < B; b += NW) {
        FC fc;
        fc.setup(TW2, lane);
        const int ib = b % NS;
        const size_t col0 = ((size_t)b * n1 + x1) * N2;
        double2 v[RC];
#pragma unroll
        for (int t = 0; t < RC; ++t) {
            const int k = fc.m + 64 * t;
            double2 val;
            if (pc.mode == 0) {
                val = h1[col0 + k];
            } else {
                val = pc.r[col0 + k];
                if (pc.mode == 2) {
                    const double2 po = pc.p_old[col0 + k];
                    if (pc.x) pc.x[col0 + k] = cadd(pc.x[col0 + k], cscale(po, alpha_prev));
                    val = cadd(val, cscale(po, beta));
                }
                pc.p[col0 + k] = val;
            }
            v[t] = cscale(val, sgn_pow(k));
            // transposed copy of the input rows within 2e of the ky edges
            if (k < 2 * g.e || k >= N2 - 2 * g.e)
                prow[((size_t)b * 4 * g.e + (k < 2 * g.e ? k : k - (N2 - 4 * g.e))) * n1 + x1] = val;
        }
        fc.template run<true>(v);
#pragma unroll
        for (int t = 0; t < RC; ++t) {
            const int n = fc.out_index(t);
            const double2 ta = cscale(TW2[(ib * n) & (N2 - 1)], sgn_pow(n));
            U[b * N2 + n] = cmul(ta, cscale(v[t], isq2 * sgn_pow(n)));
        }
    }
    __syncthreads();

    // ---- per-lane constants (tau_i u stays in shared memory: U[(s,i)][m + ML q])
    double2 acc[L][TQ];
#pragma unroll
    for (int s = 0; s < L; ++s)
#pragma unroll
        for (int q = 0; q < TQ; ++q) acc[s][q] = cmk(0.0, 0.0);
    const double2* Ui = U + i * N2 + m;
    double2 w[8];
    double sg[8];
#pragma unroll
    for (int st = 0; st < LOGM; ++st) {
        const int h = 1 << st;
        const bool upper = (m & h) == 0;
        sg[st] = upper ? 1.0 : -1.0;
        w[st] = upper ? cmk(1.0, 0.0) : twM[(m & (h - 1)) * (M / (2 * h))];
    }
    const double2 wr = MR == 2 ? twM[m] : cmk(1.0, 0.0);        // the in-register stage's twiddle w_M^m
    const int kb = (int)(__brev((unsigned)m) >> (32 - LOGM));   // this lane's bin of the lane transform
    double2 th[L][MR];                                          // CAIPI phase of register j's bin MR kb + j
#pragma unroll
    for (int s = 0; s < L; ++s)
#pragma unroll
        for (int j = 0; j < MR; ++j) th[s][j] = theta[s * N2 + i + NS * (MR * kb + j)];

    // ---- coil loop (indices past Nc are clamped and their fold is zeroed)
    const int per_iter = CG * G;
    const int iters = (Nc + per_iter - 1) / per_iter;
    const int lane_off = x1 * N2 + m;
    const int slice_stride = Nc * n1 * N2, coil_stride = n1 * N2;
#pragma unroll 1
    for (int it = 0; it < iters; ++it) {
        const int c = (it * CG + cg) * G + grp;
        const double live = (c < Nc) ? 1.0 : 0.0;
        const int cbase = lane_off + min(c, Nc - 1) * coil_stride;
        double2 sc[L][TQ];
#pragma unroll
        for (int s = 0; s < L; ++s)
#pragma unroll
            for (int q = 0; q < TQ; ++q) sc[s][q] = ST[cbase + s * slice_stride + ML * q];
        // fold: f[s][j] = sum over the positions q = j (mod MR) of S u
        double2 f[L * MR];
#pragma unroll
        for (int s = 0; s < L; ++s)
#pragma unroll
            for (int j = 0; j < MR; ++j) {
                double2 a = cmk(0.0, 0.0);
#pragma unroll
                for (int q = j; q < TQ; q += MR) a = cfma(sc[s][q], Ui[s * NS * N2 + ML * q], a);
                f[s * MR + j] = cscale(a, live);
            }
        if constexpr (MR == 2) {   // first decimation-in-frequency stage, in registers
#pragma unroll
            for (int s = 0; s < L; ++s) {
                const double2 a = f[2 * s], b = f[2 * s + 1];
                f[2 * s] = cadd(a, b);
                f[2 * s + 1] = cmul(csub(a, b), wr);
            }
        }
        fft_dif<ML, L * MR>(f, w, sg);
#pragma unroll
        for (int j = 0; j < MR; ++j) {
            double2 z = cmk(0.0, 0.0);
#pragma unroll
            for (int s = 0; s < L; ++s) z = cfma(th[s][j], f[s * MR + j], z);
#pragma unroll
            for (int s = 0; s < L; ++s) f[s * MR + j] = cmulc(z, th[s][j]);
        }
        fft_dit_inv<ML, L * MR>(f, w, sg);
        if constexpr (MR == 2) {   // last decimation-in-time stage of the inverse, in registers
#pragma unroll
            for (int s = 0; s < L; ++s) {
                const double2 a = f[2 * s], b = cmulc(f[2 * s + 1], wr);   // conj(w_M^m) B
                f[2 * s] = cadd(a, b);
                f[2 * s + 1] = csub(a, b);
            }
        }
#pragma unroll
        for (int s = 0; s < L; ++s)
#pragma unroll
            for (int q = 0; q < TQ; ++q) acc[s][q] = cadd(acc[s][q], cconjmul(sc[s][q], f[s * MR + q % MR]));
    }

    // ---- reduce the coil-group members of the wave
#pragma unroll
    for (int s = 0; s < L; ++s)
#pragma unroll
        for (int q = 0; q < TQ; ++q) {
            if constexpr (G >= 4) acc[s][q] = cadd(acc[s][q], lane_xor2<16>(acc[s][q]));
            if constexpr (G >= 2) acc[s][q] = cadd(acc[s][q], lane_xor2<32>(acc[s][q]));
        }
    // ---- normal-operator scaling conj(tau_i[n]) / n2, then the circular Hankel
    // term for the positions q = cg (mod CG) of this wave (output shot i):
    //   sum_j Khat[s][j][i][x][n] u_{s,j}[n]   (stored pairs j <= i; conjugate for j > i)
    const bool writer = (grp == 0);
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
        const int n = m + ML * q;
        const double2 tai = cscale(TW2[(i * n) & (N2 - 1)], sgn_pow(n));
        const bool mine = use_reg && writer && (q % CG == cg);
#pragma unroll
        for (int s = 0; s < L; ++s) {
            acc[s][q] = cscale(cmulc(acc[s][q], tai), 1.0 / (double)N2);
            if (mine) {
                double2 rg = cmk(0.0, 0.0);
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int pr = j <= i ? khat_pair(j, i) : khat_pair(i, j);
                    const size_t ko = ((size_t)(s * (NS * (NS + 1) / 2) + pr) * n1 + x1) * N2 + n;
                    double2 kv = KF32 ? c64to128(reinterpret_cast<const float2*>(Khat)[ko]) : Khat[ko];
                    kv.y = j <= i ? kv.y : -kv.y;
                    const double2 taj = cscale(TW2[(j * n) & (N2 - 1)], sgn_pow(n));
                    rg = cfma(kv, cmulc(U[(s * NS + j) * N2 + n], taj), rg);
                }
                acc[s][q] = cadd(acc[s][q], rg);
            }
        }
    }
    // ---- reduce the coil groups of a shot through shared memory, in order
    for (int k = 0; k < CG; ++k) {
        if (cg == k && writer) {
#pragma unroll
            for (int s = 0; s < L; ++s)
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int o = (s * NS + i) * N2 + m + ML * q;
                    ACC[o] = (k == 0) ? acc[s][q] : cadd(ACC[o], acc[s][q]);
                }
        }
        __syncthreads();
    }
    // ---- Re <p, output> in the image domain: sum conj(u) acc with u = conj(tau') U
    if (pc.mode != 0) {
        double dot = 0.0;
        for (int idx = tid; idx < B * N2; idx += nt) {
            const int b = idx / N2, n = idx - b * N2;
            const double2 ta = cscale(TW2[((b % NS) * n) & (N2 - 1)], sgn_pow(n));
            const double2 cu = cmul(ta, cconj(U[idx]));   // conj(u)
            const double2 a = ACC[idx];
            dot += cu.x * a.x - cu.y * a.y;
        }
        double* red = (double*)(sm + colfast_lds_total(g) - 16);
        dot = block_sum(dot, red);
        if (tid == 0) pc.pq[blockIdx.x] = dot;
    }
    // ---- centred forward DFT along ky of every sequence, back into ACC, then store
    for (int b = wave; b < B; b += NW) {
        FC fc;
        fc.setup(TW2, lane);
        double2 v[RC];
#pragma unroll
        for (int t = 0; t < RC; ++t) {
            const int x = fc.m + 64 * t;
            v[t] = cscale(ACC[b * N2 + x], sgn_pow(x));
        }
        fc.template run<false>(v);
#pragma unroll
        for (int t = 0; t < RC; ++t) {
            const int k = fc.out_index(t);
            ACC[b * N2 + k] = cscale(v[t], isq2 * sgn_pow(k));
        }
    }
    __syncthreads();
    for (int idx = tid; idx < B * N2; idx += nt) {
        const int b = idx / N2, j = idx - b * N2;
        h2[((size_t)b * n1 + x1) * N2 + j] = ACC[idx];
    }
}
