// HIP kernels of the SMS-MUSSELS IRLS solve (gfx950, FP64 arithmetic).
//
// Data flow of one application of the normal operator
//     N(p) = A^H A p + (lam/2) sum_l H_l^H(H_l(p_l) W_l)
// (SMS forward model of Fig. 1, block-Hankel lift of Eq. 8-9):
//   rows_inv_T  k-space rows -> inverse DFT along kx -> hybrid (x, ky),
//               written transposed so every x column is contiguous in ky;
//   col<NORMAL> one workgroup per x column: inverse DFT along ky (image),
//               coil loop with mask-pruned ky transforms (the interleaved mask
//               of shot i keeps ky = i mod Ns, so each coil image is folded to
//               n2/Ns points before its DFT), CAIPI phase and slice sum, the
//               adjoint chain, plus the circular part of the Hankel term as a
//               per-pixel Ns x Ns multiply in the image domain, then the
//               forward DFT along ky;
//   band_corr   exact correction of the Hankel term on the k-space band of
//               width r-1 where valid patch anchors end (direct taps);
//   rows_fwd_T  forward DFT along kx back to k-space, adds the band
//               correction and the partial <p, N p> of CG.
// Because the mask and the CAIPI phase depend on ky only, the kx transforms
// of A^H A cancel in the coil loop, so the coil loop needs only ky transforms.
#pragma once
#include "smsm_device.h"

#include <type_traits>

struct Geo {
    int n1, n2, L, Ns, Nc, r, K, nc, e, M, logn1, logn2, logM, B, nband, npairs;
    int cb;   // coils per pass of the generic column pass (1, 2 or 4: what its shared memory holds)
};

// ---------------------------------------------------------------------------
// Row passes
// ---------------------------------------------------------------------------

// ytil[i][c][x][m] = centred inverse DFT along kx of y[i][c][i + Ns m][:] at x
// (only the lines shot i acquires).  y is complex64.
__global__ void k_yrows_inv(Geo g, const float2* __restrict__ y, double2* __restrict__ ytil,
                            const double2* __restrict__ tw1, int TR) {
    extern __shared__ double2 sm[];
    const int n1 = g.n1, stride = n1 + 1;
    double2* v = sm;
    const int ic = blockIdx.y, i = ic / g.Nc, m0 = blockIdx.x * TR;
    const size_t ybase = (size_t)ic * g.n2 * n1;
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        const int mr = idx / n1, c = idx - mr * n1;
        const int j2 = i + g.Ns * (m0 + mr);
        v[mr * stride + c] = cscale(c64to128(y[ybase + (size_t)j2 * n1 + c]), sgn_pow(c));
    }
    fft_batch_lds(v, n1, g.logn1, TR, stride, tw1, true);
    const double sc = 1.0 / sqrt((double)n1);
    const size_t ob = (size_t)ic * n1 * g.M;
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        const int c = idx / TR, mr = idx - c * TR;
        ytil[ob + (size_t)c * g.M + m0 + mr] = cscale(v[mr * stride + c], sc * sgn_pow(c));
    }
}

// y[i][c][i + Ns m][:] = centred forward DFT along x of ytil[i][c][:][m]
// (the other lines of y must be zeroed by the caller).  y is complex128.
__global__ void k_yrows_fwd(Geo g, const double2* __restrict__ ytil, double2* __restrict__ y,
                            const double2* __restrict__ tw1, int TR) {
    extern __shared__ double2 sm[];
    const int n1 = g.n1, stride = n1 + 1;
    double2* v = sm;
    const int ic = blockIdx.y, i = ic / g.Nc, m0 = blockIdx.x * TR;
    const size_t ib = (size_t)ic * n1 * g.M;
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        const int c = idx / TR, mr = idx - c * TR;
        v[mr * stride + c] = cscale(ytil[ib + (size_t)c * g.M + m0 + mr], sgn_pow(c));
    }
    fft_batch_lds(v, n1, g.logn1, TR, stride, tw1, false);
    const double sc = 1.0 / sqrt((double)n1);
    const size_t yb = (size_t)ic * g.n2 * n1;
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        const int mr = idx / n1, k = idx - mr * n1;
        const int j2 = i + g.Ns * (m0 + mr);
        y[yb + (size_t)j2 * n1 + k] = cscale(v[mr * stride + k], sc * sgn_pow(k));
    }
}

// ---------------------------------------------------------------------------
// Column pass: one workgroup per x column, all slices and shots.
// ---------------------------------------------------------------------------
enum { COL_NORMAL = 0, COL_FWD = 1, COL_ADJ = 2, COL_REG = 3 };

// Shared-memory layout (offsets in double2 units) of k_col; the host sizes
// the launch with the same function.  The coil loop's fold and coil-map
// buffers (F [cb][B][M], SC [cb][L][n2]) share one region with what follows
// the loop's last barrier: the accumulator ACC [B][n2] (kept in registers
// during the loop) and the regulariser's taps A.
#define KCOL_ACC 10  // accumulator elements per thread (B n2 <= KCOL_ACC x threads; larger does not fit anyway)
#define KCOL_FOUT 8  // outputs per thread of the coil loop's transforms' odd-factor step (cb B M <= 8 x threads)
struct ColLds {
    int U, ACC, F, SC, TW2, TWM, A, red, total;
};
__host__ __device__ inline ColLds col_lds(const Geo& g) {
    ColLds c;
    const int bn = g.B * g.n2, loop = g.cb * (g.B * g.M + g.L * g.n2), taps = g.L * g.Ns * g.Ns * g.nc;
    c.U = 0;
    c.TW2 = c.U + bn;
    c.TWM = c.TW2 + g.n2;
    c.F = c.TWM + g.M;
    c.SC = c.F + g.cb * g.B * g.M;
    c.ACC = c.F;
    c.A = c.F + bn;
    c.red = c.F + (loop > bn + taps ? loop : bn + taps);
    c.total = c.red + 16;
    return c;
}

#define BAND_MAX_NC 17   // taps per filter dimension (2 r - 1) the kernels take

// Image-domain circular Hankel term of the normal operator (Eq. 8-9) for
// image column x1, added to ACC[(l, i')][n] (hybrid, before the final ky DFT):
//   ACC += sum_d2 w2^(d2 - e) sum_i A[l][i][i'][d2] u_{l,i}[n] conj(tau_i[n]),
//   A[l][i][i'][d2] = sum_d1 Kc[l][i][i'][d2][d1] w1^(d1 - e),
// w1 = e^{-2 pi i (x1 - n1/2)/n1}, w2 = e^{-2 pi i (n - n2/2)/n2} (tw1, TW2 hold
// e^{-2 pi i k/n}), U = tau u, tau_i[n] = (-1)^n TW2[i n mod n2].  Both tap
// sums run by Horner's rule in w1, w2 (one table lookup per sum instead of one
// per tap): an element costs Ns (nc + 1) complex multiply-adds.  A wave takes
// whole output rows (l, i') and a lane the ky points lane + 64 r, so a row's
// taps are wave-uniform and each is read once for up to four points.
// nc <= BAND_MAX_NC, n2 <= 256.  A holds
// L Ns Ns nc entries of shared memory.  The callers' ACC writes before the
// call are ordered by the barrier after the table build; they order the
// writes here before their next use of ACC.
SMSM_DEV void hankel_image_term(const Geo& g, int x1, const double2* U, const double2* __restrict__ tw1,
                                const double2* TW2, const double2* __restrict__ Kc, double2* A, double2* ACC,
                                const FastDiv& dn2, const FastDiv& dNs) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n1 = g.n1, n2 = g.n2, Ns = g.Ns, nc = g.nc, e = g.e;
    const int nu1 = x1 - n1 / 2;
    const double2 w1 = tw1[imod(nu1, n1)], w1e = tw1[imod(-e * nu1, n1)];
    for (int idx = tid; idx < g.L * Ns * Ns * nc; idx += nt) {
        // every workgroup reads the same Kc rows at once: issue a row's loads
        // together rather than one dependent load per tap
        const double2* kr = Kc + (size_t)idx * nc;
        double2 kv[BAND_MAX_NC];
#pragma unroll
        for (int d1 = 0; d1 < BAND_MAX_NC; ++d1)
            if (d1 < nc) kv[d1] = kr[d1];
        double2 p = cmk(0.0, 0.0);
#pragma unroll
        for (int d1 = BAND_MAX_NC - 1; d1 >= 0; --d1)
            if (d1 < nc) p = cfma(p, w1, kv[d1]);
        A[idx] = cmul(p, w1e);
    }
    __syncthreads();
    const int lane = tid & 63, nw = nt >> 6, R = (n2 + 63) >> 6;
    for (int b = tid >> 6; b < g.B; b += nw) {
        const int l = dNs.div(b), ip = b - l * Ns;
        double2 w2[4], acc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = min(lane + 64 * r, n2 - 1);   // lanes past n2 compute, never store
            w2[r] = TW2[imod(n - n2 / 2, n2)];
            acc[r] = cmk(0.0, 0.0);
        }
#pragma unroll 1
        for (int i = 0; i < Ns; ++i) {
            const double2* ar = A + (size_t)((l * Ns + i) * Ns + ip) * nc;
            double2 p[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) p[r] = cmk(0.0, 0.0);
#pragma unroll 4
            for (int d2 = nc - 1; d2 >= 0; --d2) {
                const double2 a = ar[d2];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r < R) p[r] = cfma(p[r], w2[r], a);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < R) {
                    const int n = min(lane + 64 * r, n2 - 1);
                    const int k = i * n - n2 * dn2.div(i * n);
                    const double2 u = cmulc(U[(l * Ns + i) * n2 + n], cscale(TW2[k], sgn_pow(n)));
                    acc[r] = cfma(p[r], u, acc[r]);
                }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = lane + 64 * r;
            if (r < R && n < n2) {
                const double2 w2e = TW2[imod(-e * (n - n2 / 2), n2)];
                ACC[b * n2 + n] = cadd(ACC[b * n2 + n], cmul(acc[r], w2e));
            }
        }
    }
}

// One workgroup per image column x (blockIdx.x).
//  COL_NORMAL  h2 = F_y[ sum_c S^H F_y^-1 M theta^H theta M F_y S u + (reg) ] for
//              u = F_y^-1 h1 (h1, h2 hybrid [B][n1][n2]);
//  COL_REG     only the circular Hankel term;
//  COL_FWD     ytil[i][c][x][m] = sum_l theta_l (F_y(S_{l,c} u_{l,i}))[i + Ns m];
//  COL_ADJ     h2 = F_y[ sum_c S^H F_y^-1 M theta^H ytil ] (input ytil, not h1).
// Mask pruning: with tau_i[n] = (-1)^n e^{-2 pi i i n/n2} and M = n2/Ns,
//  (F_y v)[i + Ns m] = (-1)^(i + Ns m)/sqrt(n2) * DFT_M( sum_t tau_i v [m + M t] )[m]
// and its adjoint unfolds an M-point inverse DFT back to n2 points (the
// (-1)^(Ns m) factors cancel in the normal operator).
template <int MODE>
__global__ void __launch_bounds__(512) k_col(Geo g, const double2* __restrict__ h1, double2* __restrict__ h2,
                      const double2* __restrict__ ST, const double2* __restrict__ theta,
                      const double2* __restrict__ tau, const double2* __restrict__ tw2,
                      const double2* __restrict__ twM, const double2* __restrict__ tw1,
                      const double2* __restrict__ Kc, int use_reg, double2* __restrict__ ytil) {
    extern __shared__ double2 sm[];
    const ColLds lay = col_lds(g);
    const int n1 = g.n1, n2 = g.n2, B = g.B, M = g.M, Ns = g.Ns, L = g.L, Nc = g.Nc;
    const int x1 = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    double2* U = sm + lay.U;
    double2* ACC = sm + lay.ACC;
    double2* F = sm + lay.F;
    double2* SC = sm + lay.SC;
    double2* TW2 = sm + lay.TW2;
    double2* TWM = sm + lay.TWM;
    double2* A = sm + lay.A;
    const double isq2 = 1.0 / sqrt((double)n2);
    const FastDiv dn2(n2), dM(M), dB(B), dNs(Ns), dL(L);   // index arithmetic (operands below 2^16)

    for (int k = tid; k < n2; k += nt) TW2[k] = tw2[k];
    for (int k = tid; k < M; k += nt) TWM[k] = twM[k];

    if (MODE != COL_ADJ) {
        // image column u = centred inverse DFT along ky; stored as tau_i * u
        for (int idx = tid; idx < B * n2; idx += nt) {
            const int b = dn2.div(idx), j = idx - b * n2;
            U[idx] = cscale(h1[((size_t)b * n1 + x1) * n2 + j], sgn_pow(j));
        }
        fft_batch_lds(U, n2, g.logn2, B, n2, TW2, true);
        for (int idx = tid; idx < B * n2; idx += nt) {
            const int b = dn2.div(idx), n = idx - b * n2, i = b - dNs.div(b) * Ns;
            U[idx] = cmul(tau[i * n2 + n], cscale(U[idx], isq2 * sgn_pow(n)));
        }
    }
    // the coil loop's accumulator: each thread's elements tid + k nt, in
    // registers (ACC shares the loop's buffers); the regulariser alone starts
    // from zero in ACC
    double2 accv[KCOL_ACC];
#pragma unroll
    for (int k = 0; k < KCOL_ACC; ++k) accv[k] = cmk(0.0, 0.0);
    if (MODE == COL_REG)
        for (int idx = tid; idx < B * n2; idx += nt) ACC[idx] = cmk(0.0, 0.0);
    __syncthreads();

    if (MODE != COL_REG) {
        // cb coils per pass (the barriers of a pass cover them all); their
        // corrections reach ACC in coil order, as one coil per pass would
        const int cb = g.cb;
        for (int c0 = 0; c0 < Nc; c0 += cb) {
            const int ncb = min(cb, Nc - c0);
            for (int idx = tid; idx < ncb * L * n2; idx += nt) {
                const int cl = dn2.div(idx), n = idx - cl * n2, cc = dL.div(cl), l = cl - cc * L;
                SC[idx] = ST[(((size_t)l * Nc + c0 + cc) * n1 + x1) * n2 + n];
            }
            __syncthreads();
            if (MODE == COL_ADJ) {
                // F[c][(l,i)][m] = conj(theta_l[i + Ns m]) * ytil[i][c][x][m]
                for (int idx = tid; idx < ncb * B * M; idx += nt) {
                    const int cb_ = dM.div(idx), m = idx - cb_ * M, cc = dB.div(cb_), b = cb_ - cc * B, l = dNs.div(b),
                              i = b - l * Ns;
                    const double2 yv = ytil[(((size_t)i * Nc + c0 + cc) * n1 + x1) * M + m];
                    F[idx] = cscale(cmulc(yv, theta[l * n2 + i + Ns * m]), sgn_pow(Ns * m));
                }
            } else {
                // fold: F[c][(l,i)][m] = sum_t S_{l,c}[m + M t] * (tau_i u_{l,i})[m + M t]
                for (int idx = tid; idx < ncb * B * M; idx += nt) {
                    const int cb_ = dM.div(idx), m = idx - cb_ * M, cc = dB.div(cb_), b = cb_ - cc * B, l = dNs.div(b);
                    const double2* scl = SC + (cc * L + l) * n2;
                    double2 f = cmk(0.0, 0.0);
                    for (int t = 0; t < Ns; ++t) {
                        const int n = m + M * t;
                        f = cfma(scl[n], U[b * n2 + n], f);
                    }
                    F[idx] = f;
                }
                fft_batch_lds<KCOL_FOUT>(F, M, g.logM, ncb * B, M, TWM, false);
                if (MODE == COL_FWD) {
                    for (int idx = tid; idx < ncb * Ns * M; idx += nt) {
                        const int cim = dM.div(idx), m = idx - cim * M, cc = dNs.div(cim), i = cim - cc * Ns, j = i + Ns * m;
                        const double2* fc = F + cc * B * M;
                        double2 z = cmk(0.0, 0.0);
                        for (int l = 0; l < L; ++l) z = cfma(theta[l * n2 + j], fc[(l * Ns + i) * M + m], z);
                        ytil[(((size_t)i * Nc + c0 + cc) * n1 + x1) * M + m] = cscale(z, isq2 * sgn_pow(i + Ns * m));
                    }
                    __syncthreads();
                    continue;
                }
                // slice sum with CAIPI phase, then back to every slice
                for (int idx = tid; idx < ncb * Ns * M; idx += nt) {
                    const int cim = dM.div(idx), m = idx - cim * M, cc = dNs.div(cim), i = cim - cc * Ns, j = i + Ns * m;
                    double2* fc = F + cc * B * M;
                    double2 z = cmk(0.0, 0.0);
                    for (int l = 0; l < L; ++l) z = cfma(theta[l * n2 + j], fc[(l * Ns + i) * M + m], z);
                    for (int l = 0; l < L; ++l) fc[(l * Ns + i) * M + m] = cmulc(z, theta[l * n2 + j]);
                }
            }
            fft_batch_lds<KCOL_FOUT>(F, M, g.logM, ncb * B, M, TWM, true);
            // unfold and accumulate conj(S) * g[n mod M], coil by coil
#pragma unroll
            for (int k = 0; k < KCOL_ACC; ++k) {
                const int idx = tid + k * nt;
                if (idx < B * n2) {
                    const int b = dn2.div(idx), n = idx - b * n2, l = dNs.div(b), nm = n - dM.div(n) * M;
                    double2 acc = accv[k];
                    for (int cc = 0; cc < ncb; ++cc)
                        acc = cadd(acc, cconjmul(SC[(cc * L + l) * n2 + n], F[(cc * B + b) * M + nm]));
                    accv[k] = acc;
                }
            }
            __syncthreads();
        }
        if (MODE == COL_FWD) return;
        // the accumulator into ACC, over the loop's buffers (the last pass
        // ended with a barrier); each thread reads back only its own elements
        // below, so no barrier is needed before that
#pragma unroll
        for (int k = 0; k < KCOL_ACC; ++k) {
            const int idx = tid + k * nt;
            if (idx < B * n2) ACC[idx] = accv[k];
        }
        // normal: conj(tau_i[n]) / n2 ; adjoint: (-1)^i conj(tau_i[n]) / sqrt(n2)
        for (int idx = tid; idx < B * n2; idx += nt) {
            const int b = dn2.div(idx), n = idx - b * n2, i = b - dNs.div(b) * Ns;
            const double s = (MODE == COL_ADJ) ? isq2 * sgn_pow(i) : 1.0 / (double)n2;
            ACC[idx] = cscale(cmulc(ACC[idx], tau[i * n2 + n]), s);
        }
    }

    if (MODE != COL_ADJ && use_reg) hankel_image_term(g, x1, U, tw1, TW2, Kc, A, ACC, dn2, dNs);
    __syncthreads();
    // centred forward DFT along ky
    for (int idx = tid; idx < B * n2; idx += nt) {
        const int n = idx % n2;
        ACC[idx] = cscale(ACC[idx], sgn_pow(n));
    }
    fft_batch_lds(ACC, n2, g.logn2, B, n2, TW2, false);
    for (int idx = tid; idx < B * n2; idx += nt) {
        const int b = dn2.div(idx), j = idx - b * n2;
        h2[((size_t)b * n1 + x1) * n2 + j] = cscale(ACC[idx], isq2 * sgn_pow(j));
    }
}

// ---------------------------------------------------------------------------
// Hankel term on the band (pixels within e = r-1 of an edge): exact minus
// circular.
//
// The circular term sums over every anchor a (mod n); the exact one only over
// anchors whose r x r patch does not wrap (a2 < n2-e and a1 < n1-e).  At pixel
// q the wrapping anchors are a = q - b' for b' in I2(q2) x [0,r) union
// [0,r) x I1(q1), where I2(q2) (I1(q1)) holds the b2' (b1') for which q2 - b2'
// (q1 - b1') lands in the last e rows (columns) mod n; it is empty unless q2
// (q1) lies within e of an edge.  By inclusion-exclusion the correction is
//   row(q) + col(q) + cross(q)
//   row(q)   = sum_d Drow[class of q2][d] p[q + d]        (b' in I2 x [0,r))
//   col(q)   = sum_d Dcol[class of q1][d] p[q + d]        (b' in [0,r) x I1)
//   cross(q) = sum_d Dx[q][d] p[q + d]                    (b' in I2 x I1, lam/2 > 0)
// The cross term only exists at the 4 e^2 corner pixels (both I2 and I1
// non-empty).  A row table serves a whole band row and a column table a
// whole band column, corners included; only the small cross part needs a
// table per corner pixel.
// ---------------------------------------------------------------------------
// Side tables (side s: 0 top, 1 bottom, 2 left, 3 right; delta = distance of
// the line from its edge, 0..e-1), output shot i' innermost:
//   Dside[l][s e + delta][i][d2][d1][i'] = -(lam/2) sum_{b' in X, b'+d in [0,r)^2} W[(i, b'+d), (i', b')]
//   X(top, delta)  = {b2' > delta} x [0,r)     X(bottom, delta) = {b2' <= delta} x [0,r)
//   X(left, delta) = [0,r) x {b1' > delta}     X(right, delta)  = [0,r) x {b1' <= delta}
// the cross tables of the corner pixels (numbered corner * e^2 + row * e +
// column, corner bit 0 = bottom, bit 1 = right)
//   Dx[l][corner pixel][i][d2][d1][i'] = (lam/2) sum_{b' in I2 x I1, b'+d in [0,r)^2} W[(i, b'+d), (i', b')]
// and the taps of the circular term (used in the image domain)
//   Kc[l][i][i'][d2][d1] = (lam/2) sum_{b'} W[(i, b'+d), (i', b')].
// f32: Dx is written as complex64 (same element index), the mixed-precision form.
__global__ void k_band_tables(Geo g, const double2* __restrict__ W, double half_lam,
                              double2* __restrict__ Kc, double2* __restrict__ Dside, double2* __restrict__ Dx,
                              int f32) {
    const int nc = g.nc, r = g.r, Ns = g.Ns, K = g.K, e = g.e, nsd = 4 * e + 4 * e * e + 1;
    const long total = (long)g.L * nsd * Ns * Ns * nc * nc;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        long t = idx;
        const int ip = t % Ns; t /= Ns;
        const int d1 = t % nc; t /= nc;
        const int d2 = t % nc; t /= nc;
        const int i = t % Ns; t /= Ns;
        const int sd = t % nsd; t /= nsd;
        const int l = (int)t;
        const int dd2 = d2 - e, dd1 = d1 - e;
        int lo2 = 0, hi2 = e, lo1 = 0, hi1 = e;    // b' ranges, inclusive
        if (sd < 4 * e) {
            const int side = sd / e, dl = sd - side * e;
            if (side == 0) lo2 = dl + 1;
            else if (side == 1) hi2 = dl;
            else if (side == 2) lo1 = dl + 1;
            else hi1 = dl;
        } else if (sd < 4 * e + 4 * e * e) {
            const int cp = sd - 4 * e, corner = cp / (e * e), px = cp - corner * e * e;
            const int rr = px / e, cc = px - rr * e;
            if (corner & 1) hi2 = rr; else lo2 = rr + 1;
            if (corner & 2) hi1 = cc; else lo1 = cc + 1;
        }
        lo2 = max(lo2, -dd2); hi2 = min(hi2, e - dd2);
        lo1 = max(lo1, -dd1); hi1 = min(hi1, e - dd1);
        const double2* Wl = W + (size_t)l * K * K;
        double2 acc = cmk(0.0, 0.0);
        for (int bp2 = lo2; bp2 <= hi2; ++bp2)
            for (int bp1 = lo1; bp1 <= hi1; ++bp1) {
                const int row = (i * r + bp2 + dd2) * r + bp1 + dd1;
                const int col = (ip * r + bp2) * r + bp1;
                acc = cadd(acc, Wl[(size_t)row * K + col]);
            }
        if (sd == nsd - 1)
            Kc[((((size_t)l * Ns + i) * Ns + ip) * nc + d2) * nc + d1] = cscale(acc, half_lam);
        else if (sd < 4 * e)
            Dside[(((((size_t)l * 4 * e + sd) * Ns + i) * nc + d2) * nc + d1) * Ns + ip] = cscale(acc, -half_lam);
        else {
            const size_t o = (((((size_t)l * 4 * e * e + sd - 4 * e) * Ns + i) * nc + d2) * nc + d1) * Ns + ip;
            const double2 v = cscale(acc, half_lam);
            if (f32) reinterpret_cast<float2*>(Dx)[o] = make_float2((float)v.x, (float)v.y);
            else Dx[o] = v;
        }
    }
}

// Band kernel, working on p in the hybrid layout (x image, ky k-space):
// one workgroup (64 Ns threads) per (work item, slice l = blockIdx.y).
//
// Row items (2e band rows x chunks of 64 x): along kx a band-row correction
// is a circular convolution of rows of p, which the kx inverse transform
// turns into a product: with Dhat[l][row][i][d2][i'][x] the x-transform of
// the row side table over d1 (built once per IRLS step),
//   crow[l Ns + i'][row][x] = sum_{i,d2} Dhat[..][x] p_i[x][ky_row + d2 - e],
// the correction of that band row already in the hybrid layout, with p read
// from its transposed band-row copy prow (contiguous x).  Thread = (output
// shot i' = wave, x = lane).
//
// Column items: BAND_SEG consecutive ky of one band column (all n2 rows) and
// a share of the 2r-1 tap columns (band_ds shares, summed where the
// correction is injected).  The natural columns of p within 2e of the kx
// edges (pcol, from k_band_extract) are staged in shared memory; wave w
// takes input shot i = w, lane = pixel, and accumulates all Ns output
// shots, with the column side table wave-uniform through the scalar cache.
//   ccol[share][l Ns + i'][column line][ky]   (natural, band column)
//
// Corner items: one corner pixel q; the Ns (2r-1)^2 taps of its cross table
// are spread over the threads (all output shots per thread), then summed by
// fixed-order block reductions: ccorner[l Ns + i'][corner pixel] (natural).
//
// Every workgroup also writes its share of Re <p, correction> (the band part
// of Re <p, N p>) to part[blockIdx.y * gridDim.x + blockIdx.x].
#define BAND_SEG 64
#define BAND_MAX_DS 4
#define BAND_STAGE 8      // staged patch entries per thread and pass
__host__ __device__ inline int band_segs(int len) { return (len + BAND_SEG - 1) / BAND_SEG; }
// shares of the tap columns (more workgroups for the same work: finer balance)
__host__ __device__ inline int band_ds(int Ns, int nc) {
    const int d = Ns >= 8 ? 2 : BAND_MAX_DS;   // measured best at 4 shots, r = 7
    return d < nc ? d : nc;
}
__host__ __device__ inline int band_col_items(const Geo& g) {
    return 2 * g.e * band_segs(g.n2) * band_ds(g.Ns, g.nc);
}
__host__ __device__ inline int band_row_items(const Geo& g) { return 2 * g.e * ((g.n1 + 63) / 64); }
__host__ __device__ inline int band_items(const Geo& g) {
    return band_col_items(g) + band_row_items(g) + 4 * g.e * g.e;
}
// shared memory of a column item: the p patch (reused for the cross-shot
// reduction afterwards)
__host__ __device__ inline size_t band_patch_len(const Geo& g) {
    const int ds = band_ds(g.Ns, g.nc);
    return (size_t)g.Ns * ((g.nc + ds - 1) / ds) * (BAND_SEG + 2 * g.e);
}
__host__ __device__ inline size_t band_lds_bytes(const Geo& g) {
    const size_t red = (size_t)g.Ns * g.Ns * BAND_SEG;
    const size_t m = band_patch_len(g) > red ? band_patch_len(g) : red;
    return (m > 8 ? m : 8) * sizeof(double2);
}
// slot of line k (within 2e of an edge of a length-n axis) in the band copies
// pcol (natural kx columns) and prow (hybrid ky rows)
SMSM_HD inline int band_pcol(int k, int n, int e) { return k < 2 * e ? k : k - (n - 4 * e); }

struct BandArgs {
    Geo g;
    const double2* pcol;    // natural columns of p within 2e of the kx edges [B][4e][n2]
    const double2* prow;    // hybrid rows of p within 2e of the ky edges, transposed [B][4e][n1]
    const double2* Dside;   // side tables (the column sides 2, 3 are used here)
    const double2* Dhat;    // row tables transformed along x [L][2e][Ns][nc][Ns][n1]
    const double2* Dx;      // corner cross tables
    double2* crow;          // [B][2e][n1], hybrid
    double2* ccol;          // [ds][B][2e][n2], natural
    double2* ccorner;       // [B][4e^2], natural
    double* part;           // Re <p, correction> per workgroup
};

template <int NC, int NS>
SMSM_DEV void band_col_sum(const double2* __restrict__ Pw, int PP, const double2* Dg, int nr,
                           double2 (&acc)[NS]) {
    // Pw: patch of this wave's shot at (first tap column of the share, this
    // lane's pixel); Dg: the side table of this wave's shot at the share's
    // first tap column, [d2][d1][i'] in global memory, read through the
    // constant address space (wave-uniform scalar loads)
    const __attribute__((address_space(4))) double* D4 =
        (const __attribute__((address_space(4))) double*)(uintptr_t)Dg;
    for (int rr = 0; rr < nr; ++rr) {
        const double2* Pr = Pw + rr * PP;
        double2 pv[NC];
#pragma unroll
        for (int dp = 0; dp < NC; ++dp) pv[dp] = Pr[dp];
#pragma unroll
        for (int dp = 0; dp < NC; ++dp) {
            const int o = 2 * ((dp * NC + rr) * NS);
#pragma unroll
            for (int ip = 0; ip < NS; ++ip) acc[ip] = cfma(cmk(D4[o + 2 * ip], D4[o + 2 * ip + 1]), pv[dp], acc[ip]);
        }
    }
}

// TF32: Dhat and Dx are stored complex64 (the mixed-precision form) and
// widened to FP64 on load.
template <int NC, int NS, bool TF32 = false>
__global__ void __launch_bounds__(64 * NS) k_band_hyb(BandArgs a) {
    extern __shared__ double2 sm[];
    __shared__ double red[16];
    const Geo& g = a.g;
    const int e = g.e, r = g.r, n1 = g.n1, n2 = g.n2, B = g.B;
    const int l = blockIdx.y, item = blockIdx.x;
    const int ncol = band_col_items(g), nrow = band_row_items(g);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double contrib = 0.0;
    if (item < ncol) {
        const int ds = band_ds(NS, NC);
        const int nseg = band_segs(n2);
        int it = item;
        const int part = it % ds;
        it /= ds;
        const int seg = it % nseg, line = it / nseg;          // column line 0..2e-1
        const int delta = line < e ? line : line - e;
        const int side = 2 + (line < e ? 0 : 1);
        const int lc = line < e ? delta : n1 - e + delta;     // kx of the line
        const int pos0 = seg * BAND_SEG;
        const int npos = min(BAND_SEG, n2 - pos0);
        const int dl0 = part * NC / ds, dl1 = (part + 1) * NC / ds, nr = dl1 - dl0;
        const int PP = BAND_SEG + 2 * e;
        // p at this thread's output (output shot = wave, pixel = lane), for Re <p, correction>
        const double2 pout = a.pcol[((size_t)(l * NS + w) * 4 * e + band_pcol(lc, n1, e)) * n2 + pos0 +
                                    min(lane, npos - 1)];
        // stage sm[i][rr][pp] = p_i at kx = lc - e + dl0 + rr, ky = pos0 - e + pp
        // (wrapped); at most BAND_STAGE entries per thread, all loads issued
        // together (threads past the end reload the last entry)
        const int tot = NS * nr * PP;
        // the wrap of the staged lines: a mask for power-of-two sizes (the same
        // for every thread, so the two copies of the loop are a uniform branch)
        auto stage = [&](auto pow2) {
            for (int base = threadIdx.x; base < tot; base += BAND_STAGE * blockDim.x) {
                double2 v[BAND_STAGE];
#pragma unroll
                for (int u = 0; u < BAND_STAGE; ++u) {
                    const int i0 = base + u * blockDim.x, idx = i0 < tot ? i0 : tot - 1;
                    const int i = idx / (nr * PP), rem = idx - i * nr * PP;
                    const int rr = rem / PP, pp = rem - rr * PP;
                    const int kx = decltype(pow2)::value ? (lc - e + dl0 + rr) & (n1 - 1) : wrap1(lc - e + dl0 + rr, n1);
                    const int ky = decltype(pow2)::value ? (pos0 - e + pp) & (n2 - 1) : wrap1(pos0 - e + pp, n2);
                    v[u] = a.pcol[((size_t)(l * NS + i) * 4 * e + band_pcol(kx, n1, e)) * n2 + ky];
                }
#pragma unroll
                for (int u = 0; u < BAND_STAGE; ++u) {
                    const int i0 = base + u * blockDim.x;
                    sm[i0 < tot ? i0 : tot - 1] = v[u];
                }
            }
        };
        if ((n1 & (n1 - 1)) == 0 && (n2 & (n2 - 1)) == 0) stage(std::true_type{});
        else stage(std::false_type{});
        const double2* Dsrc = a.Dside + ((size_t)l * 4 * e + side * e + delta) * NS * NC * NC * NS;
        __syncthreads();
        const double2* Pw = sm + (size_t)w * nr * PP + min(lane, npos - 1);
        double2 acc[NS];
#pragma unroll
        for (int ip = 0; ip < NS; ++ip) acc[ip] = cmk(0.0, 0.0);
        band_col_sum<NC, NS>(Pw, PP, Dsrc + ((size_t)w * NC * NC + dl0) * NS, nr, acc);
        __syncthreads();
#pragma unroll
        for (int ip = 0; ip < NS; ++ip) sm[((size_t)w * NS + ip) * BAND_SEG + lane] = acc[ip];
        __syncthreads();
        {   // one output per thread: shot ip = wave, pixel px = lane
            const int ip = w, px = lane;
            const size_t o = (((size_t)l * NS + ip) * 2 * e + line) * n2 + pos0 + px, pstride = (size_t)B * 2 * e * n2;
            if (px < npos) {
                double2 s = cmk(0.0, 0.0);
#pragma unroll
                for (int i = 0; i < NS; ++i) s = cadd(s, sm[((size_t)i * NS + ip) * BAND_SEG + px]);
                a.ccol[part * pstride + o] = s;
                contrib = pout.x * s.x + pout.y * s.y;
            }
        }
    } else if (item < ncol + nrow) {
        const int ri = item - ncol, nxc = (n1 + 63) / 64;
        const int line = ri / nxc, x = (ri - line * nxc) * 64 + lane;
        const int ky = line < e ? line : n2 - 2 * e + line;
        const int ip = w;
        if (x < n1) {
            const double2 pout = a.prow[((size_t)(l * NS + ip) * 4 * e + band_pcol(ky, n2, e)) * n1 + x];
            const size_t dh0 = ((size_t)(l * 2 * e + line) * NS * NC * NS) * n1 + x;
            double2 s = cmk(0.0, 0.0);
            // one input shot per round, its 2 NC loads issued as one batch
            // (two shots per round need more registers than the column items
            // sharing this kernel can spare)
            constexpr int IR = 1;
            for (int i0 = 0; i0 < NS; i0 += IR) {
                double2 dv[IR][NC], pv[IR][NC];
#pragma unroll
                for (int u = 0; u < IR; ++u) {
                    const int i = i0 + u;
                    const double2* pri = a.prow + (size_t)(l * NS + i) * 4 * e * n1 + x;
#pragma unroll
                    for (int d2 = 0; d2 < NC; ++d2) {
                        const size_t o = dh0 + (((size_t)i * NC + d2) * NS + ip) * n1;
                        dv[u][d2] = TF32 ? c64to128(reinterpret_cast<const float2*>(a.Dhat)[o]) : a.Dhat[o];
                        pv[u][d2] = pri[(size_t)band_pcol(wrap1(ky + d2 - e, n2), n2, e) * n1];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < IR; ++u)
#pragma unroll
                    for (int d2 = 0; d2 < NC; ++d2) s = cfma(dv[u][d2], pv[u][d2], s);
            }
            a.crow[((size_t)(l * NS + ip) * 2 * e + line) * n1 + x] = s;
            contrib = pout.x * s.x + pout.y * s.y;
        }
    } else {
        const int cp = item - ncol - nrow;
        const int corner = cp / (e * e), px = cp - corner * e * e;
        const int rr = px / e, cc = px - rr * e;
        const int q2 = ((corner & 1) ? n2 - e : 0) + rr, q1 = ((corner & 2) ? n1 - e : 0) + cc;
        const size_t dc0 = ((size_t)l * 4 * e * e + cp) * NS * NC * NC * NS;
        const int cq = band_pcol(q1, n1, e);
        double2 pq[NS];
#pragma unroll
        for (int ip = 0; ip < NS; ++ip) pq[ip] = a.pcol[((size_t)(l * NS + ip) * 4 * e + cq) * n2 + q2];
        double2 acc[NS];
#pragma unroll
        for (int ip = 0; ip < NS; ++ip) acc[ip] = cmk(0.0, 0.0);
        // the taps spread over the threads, all loads of a thread issued together
        constexpr int nt = NS * NC * NC, TPB = 64 * NS, IT = (nt + TPB - 1) / TPB;
        double2 pv[IT], dc[IT][NS];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int t0 = threadIdx.x + it * TPB, t = t0 < nt ? t0 : nt - 1;
            const int i = t / (NC * NC), d = t - i * NC * NC, d2 = d / NC, d1 = d - d2 * NC;
            const int kx = wrap1(q1 - e + d1, n1), ky = wrap1(q2 - e + d2, n2);
            pv[it] = a.pcol[((size_t)(l * NS + i) * 4 * e + band_pcol(kx, n1, e)) * n2 + ky];
#pragma unroll
            for (int ip = 0; ip < NS; ++ip) {
                const size_t o = dc0 + (size_t)t * NS + ip;
                dc[it][ip] = TF32 ? c64to128(reinterpret_cast<const float2*>(a.Dx)[o]) : a.Dx[o];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const double live = threadIdx.x + it * TPB < nt ? 1.0 : 0.0;
#pragma unroll
            for (int ip = 0; ip < NS; ++ip) acc[ip] = cfma(dc[it][ip], cscale(pv[it], live), acc[ip]);
        }
        // all 2 NS sums in one exchange
        double v[2 * NS];
#pragma unroll
        for (int ip = 0; ip < NS; ++ip) {
            v[2 * ip] = acc[ip].x;
            v[2 * ip + 1] = acc[ip].y;
        }
        block_sum_n<2 * NS>(v, (double*)sm);   // 2 NS NS doubles; the corner items use no other shared memory
        if (threadIdx.x == 0) {
#pragma unroll
            for (int ip = 0; ip < NS; ++ip) {
                a.ccorner[((size_t)l * NS + ip) * 4 * e * e + cp] = cmk(v[2 * ip], v[2 * ip + 1]);
                contrib += pq[ip].x * v[2 * ip] + pq[ip].y * v[2 * ip + 1];
            }
        }
    }
    contrib = block_sum(contrib, red);
    if (threadIdx.x == 0) a.part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = contrib;
}

// Band kernel for (2r-1, Ns); null when the pair is outside what the plan
// accepts (Ns r^2 <= 256, 2r-1 <= BAND_MAX_NC).
typedef void (*BandFn)(BandArgs);
template <int NS, bool TF32>
inline BandFn band_fn_ns(int nc) {
    switch (nc) {
        case 3: return &k_band_hyb<3, NS, TF32>;
        case 5: return &k_band_hyb<5, NS, TF32>;
        case 7: return &k_band_hyb<7, NS, TF32>;
        case 9: return &k_band_hyb<9, NS, TF32>;
        case 11: return NS <= 4 ? &k_band_hyb<11, (NS <= 4 ? NS : 4), TF32> : nullptr;
        case 13: return NS <= 4 ? &k_band_hyb<13, (NS <= 4 ? NS : 4), TF32> : nullptr;
        case 15: return NS <= 4 ? &k_band_hyb<15, (NS <= 4 ? NS : 4), TF32> : nullptr;
        case 17: return NS <= 2 ? &k_band_hyb<17, (NS <= 2 ? NS : 2), TF32> : nullptr;
        default: return nullptr;
    }
}
// tf32: the instance reading complex64 tables
inline BandFn band_fn(int nc, int ns, bool tf32 = false) {
    switch (ns) {
        case 1: return tf32 ? band_fn_ns<1, true>(nc) : band_fn_ns<1, false>(nc);
        case 2: return tf32 ? band_fn_ns<2, true>(nc) : band_fn_ns<2, false>(nc);
        case 4: return tf32 ? band_fn_ns<4, true>(nc) : band_fn_ns<4, false>(nc);
        case 8: return tf32 ? band_fn_ns<8, true>(nc) : band_fn_ns<8, false>(nc);
        default: return nullptr;
    }
}

// Row tables along x: Dhat[l][row][i][d2][i'][x] = sum_d1 Drow[l][row][i][d2][d1][i']
// e^{-2 pi i (d1 - e)(x - n1/2)/n1}, rows 0..e-1 top and e..2e-1 bottom
// (side tables 0 and 1).  One workgroup per (l, row, i, d2) with its taps and
// the kx twiddles in shared memory; thread = x, all i'.
// f32: written as complex64 (same element index), the mixed-precision form.
template <bool POW2>
__global__ void __launch_bounds__(256) k_band_rowhat(Geo g, const double2* __restrict__ Dside,
                                                     const double2* __restrict__ tw1, double2* __restrict__ Dhat,
                                                     int f32) {
    __shared__ double2 T1[256];
    __shared__ double2 DR[BAND_MAX_NC * 8];   // [d1][i'], Ns <= 8
    const int n1 = g.n1, Ns = g.Ns, nc = g.nc, e = g.e;
    const int lrid = blockIdx.x;                            // ((l * 2e + row) * Ns + i) * nc + d2
    // rows 0..2e-1 are the side tables 0 (top) and 1 (bottom), in that order
    const int d2 = lrid % nc, i = (lrid / nc) % Ns, row = (lrid / (nc * Ns)) % (2 * e), l = lrid / (nc * Ns * 2 * e);
    const double2* dr = Dside + ((((size_t)l * 4 * e + row) * Ns + i) * nc + d2) * nc * Ns;
    for (int t = threadIdx.x; t < n1; t += blockDim.x) T1[t] = tw1[t];
    for (int t = threadIdx.x; t < nc * Ns; t += blockDim.x) DR[t] = dr[t];
    __syncthreads();
    const size_t out0 = (size_t)lrid * Ns * n1;
    for (int x = threadIdx.x; x < n1; x += blockDim.x) {
        for (int ip = 0; ip < Ns; ++ip) {
            double2 s = cmk(0.0, 0.0);
            for (int d1 = 0; d1 < nc; ++d1) {
                const int ph = (d1 - e) * (x - n1 / 2);
                s = cfma(DR[d1 * Ns + ip], T1[POW2 ? ph & (n1 - 1) : imod(ph, n1)], s);
            }
            if (f32) reinterpret_cast<float2*>(Dhat)[out0 + (size_t)ip * n1 + x] = make_float2((float)s.x, (float)s.y);
            else Dhat[out0 + (size_t)ip * n1 + x] = s;
        }
    }
}

// Band corrections as the hybrid-layout vector pass takes them: the row
// corrections (already transformed along kx), the natural corrections on the
// 2e band columns in ds shares, the corner cross terms, and
// finv[x][cl] = e^{+2 pi i (kx_cl - n1/2)(x - n1/2)/n1} / sqrt(n1), the kx
// inverse transform restricted to the band columns kx_cl (cl < e: cl, else
// n1 - 2e + cl); rows are 16 entries wide, zero past 2e.
struct BandInj {
    const double2* crow;
    const double2* ccol;
    const double2* ccorner;
    const double2* finv;
    int ds;
};
// ---------------------------------------------------------------------------
// Plain vector kernels (fixed grid, grid-stride).
// ---------------------------------------------------------------------------
__global__ void k_copy_c128(long n, const double2* __restrict__ a, double2* __restrict__ b) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) b[k] = a[k];
}

__global__ void k_to_c64(long n, const double2* __restrict__ a, float2* __restrict__ b) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        b[k] = make_float2((float)a[k].x, (float)a[k].y);
}

__global__ void k_zero_c128(long n, double2* __restrict__ a) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        a[k] = cmk(0.0, 0.0);
}

__global__ void k_zero_i32(long n, int* __restrict__ a) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) a[k] = 0;
}

// Coil maps c64 [L][Nc][n2][n1] -> plan layout c128 [L][Nc][n1][n2] (x-major columns; widened once).
__global__ void k_transpose_coils(int n1, int n2, long nimg, const float2* __restrict__ S,
                                  double2* __restrict__ ST) {
    const long total = nimg * n1 * n2;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long img = k / ((long)n1 * n2);
        const int rem = (int)(k - img * n1 * n2);
        const int x = rem / n2, y = rem - x * n2;
        ST[k] = c64to128(S[img * n1 * n2 + (long)y * n1 + x]);
    }
}

// eps_l = mult * sigma_l for the current IRLS step (device-side schedule).
__global__ void k_eps(int L, const double* __restrict__ sigma, double mult, double* __restrict__ eps) {
    const int l = threadIdx.x;
    if (l < L) eps[l] = mult * sigma[l];
}
