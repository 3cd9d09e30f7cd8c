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

struct Geo {
    int n1, n2, L, Ns, Nc, r, K, nc, e, M, logn1, logn2, logM, B, nband, npairs;
};

// ---------------------------------------------------------------------------
// Band of the k-space grid where the Hankel term differs from its circular
// version: rows/columns within e = r-1 of an edge.  Enumeration: the e top
// rows and e bottom rows (row-major), then the 2e edge columns of the middle
// rows (column-major, so consecutive indices share a tap class).
// ---------------------------------------------------------------------------
SMSM_DEV int band_index(const Geo& g, int t2, int t1) {
    const int e = g.e;
    if (t2 < e) return t2 * g.n1 + t1;
    if (t2 >= g.n2 - e) return (e + t2 - (g.n2 - e)) * g.n1 + t1;
    int cc;
    if (t1 < e) cc = t1;
    else if (t1 >= g.n1 - e) cc = e + t1 - (g.n1 - e);
    else return -1;
    return 2 * e * g.n1 + cc * (g.n2 - 2 * e) + (t2 - e);
}

SMSM_DEV void band_pos(const Geo& g, int idx, int& t2, int& t1) {
    const int e = g.e, top = 2 * e * g.n1;
    if (idx < top) {
        const int row = idx / g.n1;
        t1 = idx - row * g.n1;
        t2 = row < e ? row : g.n2 - e + (row - e);
    } else {
        const int k = idx - top, h = g.n2 - 2 * e;
        const int cc = k / h;
        t2 = e + (k - cc * h);
        t1 = cc < e ? cc : g.n1 - e + (cc - e);
    }
}

// Tap class of a coordinate: 0..r-2 near the low edge, r-1 interior,
// r..2r-2 near the high edge.
SMSM_DEV int band_class(int t, int n, int r) {
    if (t <= r - 2) return t;
    if (t >= n - r + 1) return r + (t - (n - r + 1));
    return r - 1;
}

// ---------------------------------------------------------------------------
// Row passes
// ---------------------------------------------------------------------------
enum { ROWS_PLAIN = 0, ROWS_CG_UPDATE = 1, ROWS_CG_FIRST = 2 };

// out[b][x][j2] = centred inverse DFT along kx of in[b][j2][:], evaluated at x.
// ROWS_CG_UPDATE: the transformed vector is p = r + beta p (beta = rr_j/rr_{j-1}
// from block partials), written back to p.  ROWS_CG_FIRST: p = r.
template <int MODE>
__global__ void k_rows_inv_T(Geo g, const double2* __restrict__ in, double2* __restrict__ out,
                             const double2* __restrict__ rvec, double2* __restrict__ pvec,
                             const double* __restrict__ pr_new, const double* __restrict__ pr_old,
                             int npart, const double2* __restrict__ tw1, int TR) {
    extern __shared__ double2 sm[];
    const int n1 = g.n1, stride = n1 + 1;
    double2* v = sm;
    double* red = (double*)(sm + TR * stride);
    const int b = blockIdx.y, j0 = blockIdx.x * TR;
    double beta = 0.0;
    if (MODE == ROWS_CG_UPDATE) {
        const double rn = sum_partials(pr_new, npart, red);
        const double ro = sum_partials(pr_old, npart, red);
        beta = (ro > 0.0) ? rn / ro : 0.0;
    }
    const size_t img = (size_t)b * g.n2 * n1;
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        const int jr = idx / n1, c = idx - jr * n1;
        const size_t o = img + (size_t)(j0 + jr) * n1 + c;
        double2 val;
        if (MODE == ROWS_PLAIN) {
            val = in[o];
        } else if (MODE == ROWS_CG_UPDATE) {
            val = cadd(rvec[o], cscale(pvec[o], beta));
            pvec[o] = val;
        } else {
            val = rvec[o];
            pvec[o] = val;
        }
        v[jr * stride + c] = cscale(val, sgn_pow(c));
    }
    fft_batch_lds(v, n1, g.logn1, TR, stride, tw1, true);
    const double sc = 1.0 / sqrt((double)n1);
    const size_t ob = (size_t)b * n1 * g.n2;
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        const int c = idx / TR, jr = idx - c * TR;
        out[ob + (size_t)c * g.n2 + j0 + jr] = cscale(v[jr * stride + c], sc * sgn_pow(c));
    }
}

// out[b][j2][:] = centred forward DFT along x of in[b][:][j2] (hybrid, transposed).
// BAND: adds corr[b][band_index] on band pixels.  CG: per-block partial of
// Re<p, out> into pq_part[block].
template <bool CG, bool BAND>
__global__ void k_rows_fwd_T(Geo g, const double2* __restrict__ in, double2* __restrict__ out,
                             const double2* __restrict__ corr, const double2* __restrict__ pvec,
                             double* __restrict__ pq_part, const double2* __restrict__ tw1, int TR) {
    extern __shared__ double2 sm[];
    const int n1 = g.n1, stride = n1 + 1;
    double2* v = sm;
    double* red = (double*)(sm + TR * stride);
    const int b = blockIdx.y, j0 = blockIdx.x * TR;
    const size_t ib = (size_t)b * n1 * g.n2;
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        const int c = idx / TR, jr = idx - c * TR;
        v[jr * stride + c] = cscale(in[ib + (size_t)c * g.n2 + j0 + jr], sgn_pow(c));
    }
    fft_batch_lds(v, n1, g.logn1, TR, stride, tw1, false);
    const double sc = 1.0 / sqrt((double)n1);
    const size_t img = (size_t)b * g.n2 * n1;
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < TR * n1; idx += blockDim.x) {
        const int jr = idx / n1, k = idx - jr * n1;
        const int j2 = j0 + jr;
        double2 val = cscale(v[jr * stride + k], sc * sgn_pow(k));
        if (BAND) {
            const int bi = band_index(g, j2, k);
            if (bi >= 0) val = cadd(val, corr[(size_t)b * g.nband + bi]);
        }
        const size_t o = img + (size_t)j2 * n1 + k;
        out[o] = val;
        if (CG) {
            const double2 pv = pvec[o];
            acc += pv.x * val.x + pv.y * val.y;
        }
    }
    if (CG) {
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) pq_part[blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

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
// the launch with the same function.
struct ColLds {
    int U, ACC, F, SC, TW2, TWM, A, red, total;
};
__host__ __device__ inline ColLds col_lds(const Geo& g) {
    ColLds c;
    c.U = 0;
    c.ACC = c.U + g.B * g.n2;
    c.F = c.ACC + g.B * g.n2;
    c.SC = c.F + g.B * g.M;
    c.TW2 = c.SC + g.L * g.n2;
    c.TWM = c.TW2 + g.n2;
    c.A = c.TWM + g.M;
    c.red = c.A + g.L * g.Ns * g.Ns * g.nc;
    c.total = c.red + 16;
    return c;
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
__global__ void k_col(Geo g, const double2* __restrict__ h1, double2* __restrict__ h2,
                      const float2* __restrict__ ST, const double2* __restrict__ theta,
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

    for (int k = tid; k < n2; k += nt) TW2[k] = tw2[k];
    for (int k = tid; k < M; k += nt) TWM[k] = twM[k];

    if (MODE != COL_ADJ) {
        // image column u = centred inverse DFT along ky; stored as tau_i * u
        for (int idx = tid; idx < B * n2; idx += nt) {
            const int b = idx / n2, j = idx - b * n2;
            U[idx] = cscale(h1[((size_t)b * n1 + x1) * n2 + j], sgn_pow(j));
        }
        fft_batch_lds(U, n2, g.logn2, B, n2, TW2, true);
        for (int idx = tid; idx < B * n2; idx += nt) {
            const int b = idx / n2, n = idx - b * n2, i = b % Ns;
            U[idx] = cmul(tau[i * n2 + n], cscale(U[idx], isq2 * sgn_pow(n)));
        }
    }
    if (MODE != COL_FWD)
        for (int idx = tid; idx < B * n2; idx += nt) ACC[idx] = cmk(0.0, 0.0);
    __syncthreads();

    if (MODE != COL_REG) {
        for (int c = 0; c < Nc; ++c) {
            for (int idx = tid; idx < L * n2; idx += nt) {
                const int l = idx / n2, n = idx - l * n2;
                SC[idx] = c64to128(ST[(((size_t)l * Nc + c) * n1 + x1) * n2 + n]);
            }
            if (MODE == COL_ADJ) {
                __syncthreads();
                // F[(l,i)][m] = conj(theta_l[i + Ns m]) * ytil[i][c][x][m]
                for (int idx = tid; idx < B * M; idx += nt) {
                    const int b = idx / M, m = idx - b * M, l = b / Ns, i = b - l * Ns;
                    const double2 yv = ytil[(((size_t)i * Nc + c) * n1 + x1) * M + m];
                    F[idx] = cscale(cmulc(yv, theta[l * n2 + i + Ns * m]), sgn_pow(Ns * m));
                }
            } else {
                __syncthreads();
                // fold: F[(l,i)][m] = sum_t S_l[m + M t] * (tau_i u_{l,i})[m + M t]
                for (int idx = tid; idx < B * M; idx += nt) {
                    const int b = idx / M, m = idx - b * M, l = b / Ns;
                    double2 f = cmk(0.0, 0.0);
                    for (int t = 0; t < Ns; ++t) {
                        const int n = m + M * t;
                        f = cfma(SC[l * n2 + n], U[b * n2 + n], f);
                    }
                    F[idx] = f;
                }
                fft_batch_lds(F, M, g.logM, B, M, TWM, false);
                if (MODE == COL_FWD) {
                    for (int idx = tid; idx < Ns * M; idx += nt) {
                        const int i = idx / M, m = idx - i * M, j = i + Ns * m;
                        double2 z = cmk(0.0, 0.0);
                        for (int l = 0; l < L; ++l) z = cfma(theta[l * n2 + j], F[(l * Ns + i) * M + m], z);
                        ytil[(((size_t)i * Nc + c) * n1 + x1) * M + m] = cscale(z, isq2 * sgn_pow(i + Ns * m));
                    }
                    __syncthreads();
                    continue;
                }
                // slice sum with CAIPI phase, then back to every slice
                for (int idx = tid; idx < Ns * M; idx += nt) {
                    const int i = idx / M, m = idx - i * M, j = i + Ns * m;
                    double2 z = cmk(0.0, 0.0);
                    for (int l = 0; l < L; ++l) z = cfma(theta[l * n2 + j], F[(l * Ns + i) * M + m], z);
                    for (int l = 0; l < L; ++l) F[(l * Ns + i) * M + m] = cmulc(z, theta[l * n2 + j]);
                }
            }
            fft_batch_lds(F, M, g.logM, B, M, TWM, true);
            // unfold and accumulate conj(S) * g[n mod M]
            for (int idx = tid; idx < B * n2; idx += nt) {
                const int b = idx / n2, n = idx - b * n2, l = b / Ns;
                ACC[idx] = cadd(ACC[idx], cconjmul(SC[l * n2 + n], F[b * M + (n & (M - 1))]));
            }
            __syncthreads();
        }
        if (MODE == COL_FWD) return;
        // normal: conj(tau_i[n]) / n2 ; adjoint: (-1)^i conj(tau_i[n]) / sqrt(n2)
        for (int idx = tid; idx < B * n2; idx += nt) {
            const int b = idx / n2, n = idx - b * n2, i = b % Ns;
            const double s = (MODE == COL_ADJ) ? isq2 * sgn_pow(i) : 1.0 / (double)n2;
            ACC[idx] = cscale(cmulc(ACC[idx], tau[i * n2 + n]), s);
        }
    }

    if (MODE != COL_ADJ && use_reg) {
        // A[l][i][i'][d2] = sum_d1 Kc[l][i][i'][d2][d1] e^{-2 pi i d1 (x - n1/2)/n1}
        const int nc = g.nc, e = g.e, nu1 = x1 - n1 / 2;
        for (int idx = tid; idx < L * Ns * Ns * nc; idx += nt) {
            const double2* kr = Kc + (size_t)idx * nc;
            double2 a = cmk(0.0, 0.0);
            for (int d1 = 0; d1 < nc; ++d1) {
                const int ph = ((d1 - e) * nu1) & (n1 - 1);
                a = cfma(kr[d1], tw1[ph], a);
            }
            A[idx] = a;
        }
        __syncthreads();
        // ACC[(l,i')][n] += sum_i sum_d2 A[l][i][i'][d2] e^{-2 pi i d2 (n - n2/2)/n2} u_{l,i}[n]
        for (int idx = tid; idx < B * n2; idx += nt) {
            const int b = idx / n2, n = idx - b * n2, l = b / Ns, ip = b - l * Ns;
            const int nu2 = n - n2 / 2;
            double2 s = cmk(0.0, 0.0);
            for (int i = 0; i < Ns; ++i) {
                const double2 u = cmulc(U[(l * Ns + i) * n2 + n], tau[i * n2 + n]);
                const double2* ar = A + ((size_t)(l * Ns + i) * Ns + ip) * nc;
                double2 kv = cmk(0.0, 0.0);
                for (int d2 = 0; d2 < nc; ++d2) kv = cfma(ar[d2], TW2[((d2 - e) * nu2) & (n2 - 1)], kv);
                s = cfma(kv, u, s);
            }
            ACC[idx] = cadd(ACC[idx], s);
        }
    }
    __syncthreads();
    // centred forward DFT along ky
    for (int idx = tid; idx < B * n2; idx += nt) {
        const int n = idx % n2;
        ACC[idx] = cscale(ACC[idx], sgn_pow(n));
    }
    fft_batch_lds(ACC, n2, g.logn2, B, n2, TW2, false);
    for (int idx = tid; idx < B * n2; idx += nt) {
        const int b = idx / n2, j = idx - b * n2;
        h2[((size_t)b * n1 + x1) * n2 + j] = cscale(ACC[idx], isq2 * sgn_pow(j));
    }
}

// ---------------------------------------------------------------------------
// Hankel term on the band: exact minus circular, with per-class tap tables.
// ---------------------------------------------------------------------------
// Tap tables from W (lam/2 folded in):
//   Kc[l][i][i'][d2][d1]             = sum_{b'} W[(i, b'+d), (i', b')]
//   D[l][c2][c1][i'][i][d2][d1]      = K^{(c2,c1)}[i][i'][d] - Kc[l][i][i'][d]
// where K^{(class)} restricts b' to the anchors valid for that band class.
__global__ void k_band_tables(Geo g, const double2* __restrict__ W, double half_lam,
                              double2* __restrict__ Kc, double2* __restrict__ D) {
    const int nc = g.nc, r = g.r, Ns = g.Ns, K = g.K;
    const long total = (long)g.L * nc * nc * Ns * Ns * nc * nc;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        long t = idx;
        const int d1 = t % nc; t /= nc;
        const int d2 = t % nc; t /= nc;
        const int i = t % Ns; t /= Ns;
        const int ip = t % Ns; t /= Ns;
        const int c1 = t % nc; t /= nc;
        const int c2 = t % nc; t /= nc;
        const int l = (int)t;
        const int dd2 = d2 - (r - 1), dd1 = d1 - (r - 1);
        // b' range of the class in each dimension
        const int lo2 = (c2 < r) ? 0 : c2 - (r - 1), hi2 = (c2 < r) ? c2 : r - 1;
        const int lo1 = (c1 < r) ? 0 : c1 - (r - 1), hi1 = (c1 < r) ? c1 : r - 1;
        const double2* Wl = W + (size_t)l * K * K;
        double2 kfull = cmk(0.0, 0.0), kcls = cmk(0.0, 0.0);
        const int a2 = max(0, -dd2), z2 = min(r - 1, r - 1 - dd2);
        const int a1 = max(0, -dd1), z1 = min(r - 1, r - 1 - dd1);
        for (int bp2 = a2; bp2 <= z2; ++bp2) {
            for (int bp1 = a1; bp1 <= z1; ++bp1) {
                const int row = (i * r + bp2 + dd2) * r + bp1 + dd1;
                const int col = (ip * r + bp2) * r + bp1;
                const double2 w = Wl[(size_t)row * K + col];
                kfull = cadd(kfull, w);
                if (bp2 >= lo2 && bp2 <= hi2 && bp1 >= lo1 && bp1 <= hi1) kcls = cadd(kcls, w);
            }
        }
        kfull = cscale(kfull, half_lam);
        kcls = cscale(kcls, half_lam);
        D[idx] = csub(kcls, kfull);
        if (c2 == r - 1 && c1 == r - 1)
            Kc[((((size_t)l * Ns + i) * Ns + ip) * nc + d2) * nc + d1] = kfull;
    }
}

// corr[(l,i')][bidx] = sum_i sum_d D[l][class][i'][i][d] p[l][i][(t + d) mod n]
__global__ void k_band_corr(Geo g, const double2* __restrict__ p, const double2* __restrict__ D,
                            double2* __restrict__ corr) {
    const int nc = g.nc, r = g.r, Ns = g.Ns, n1 = g.n1, n2 = g.n2;
    const int total = g.B * g.nband;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int b = idx / g.nband, bi = idx - b * g.nband;
    const int l = b / Ns, ip = b - l * Ns;
    int t2, t1;
    band_pos(g, bi, t2, t1);
    const int c2 = band_class(t2, n2, r), c1 = band_class(t1, n1, r);
    const double2* Dp = D + ((((size_t)l * nc + c2) * nc + c1) * Ns + ip) * (size_t)Ns * nc * nc;
    double2 s = cmk(0.0, 0.0);
    for (int i = 0; i < Ns; ++i) {
        const double2* pi = p + ((size_t)l * Ns + i) * n2 * n1;
        for (int d2 = 0; d2 < nc; ++d2) {
            const int q2 = (t2 + d2 - (r - 1)) & (n2 - 1);
            const double2* prow = pi + (size_t)q2 * n1;
            const double2* dr = Dp + ((size_t)i * nc + d2) * nc;
            for (int d1 = 0; d1 < nc; ++d1) {
                const int q1 = (t1 + d1 - (r - 1)) & (n1 - 1);
                s = cfma(dr[d1], prow[q1], s);
            }
        }
    }
    corr[idx] = s;
}

// Tiled version: one workgroup per (band tile, slice l, output shot i').
// Edge tiles cover TW = 64 pixels along one strip (top/bottom rows 0..e-1 and
// n2-e..n2-1 between the corner blocks, left/right columns likewise) and all
// e lines of the strip; wave k of the workgroup computes line k with one pixel
// per lane.  Every pixel of a line shares one tap table, so the e tables of
// the tile are staged in shared memory next to the p patch of all shots (tile
// plus an e-wide halo, wrapped, strip direction contiguous); table reads are
// broadcasts.  The four e x e corner blocks (one table per pixel) are tiles
// of their own, one pixel per lane, tables read through the cache.
#define BAND_TW 64
__host__ __device__ inline int band_edge_tiles(int len, int e) { return (len - 2 * e + BAND_TW - 1) / BAND_TW; }
__host__ __device__ inline int band_tiles_total(const Geo& g) {
    return 2 * band_edge_tiles(g.n1, g.e) + 2 * band_edge_tiles(g.n2, g.e) + 4;
}
__host__ __device__ inline size_t band_patch_elems(const Geo& g) {
    return (size_t)g.Ns * (3 * g.e) * (BAND_TW + 2 * g.e);
}
__host__ __device__ inline size_t band_lds_bytes(const Geo& g) {
    return (band_patch_elems(g) + (size_t)g.e * g.Ns * g.nc * g.nc) * sizeof(double2);
}

#define BAND_MAX_NC 17
template <int NC>
__global__ void __launch_bounds__(1024)
k_band_tile(Geo g, const double2* __restrict__ p, const double2* __restrict__ D, double2* __restrict__ corr) {
    extern __shared__ double2 sm[];
    constexpr int nc = NC, tab = NC * NC;
    const int e = g.e, r = g.r, Ns = g.Ns, n1 = g.n1, n2 = g.n2;
    const int nth = band_edge_tiles(n1, e), ntv = band_edge_tiles(n2, e);
    const int l = blockIdx.y, ip = blockIdx.z;
    const int tile = blockIdx.x;
    int kind;  // 0 top, 1 bottom, 2 left, 3 right, 4 corner
    int t2a, t1a, H, Wd;
    if (tile < 2 * nth) {
        kind = tile < nth ? 0 : 1;
        const int k = tile - (kind == 1 ? nth : 0);
        t2a = kind == 0 ? 0 : n2 - e;
        t1a = e + k * BAND_TW;
        H = e;
        Wd = min(BAND_TW, n1 - e - t1a);
    } else if (tile < 2 * nth + 2 * ntv) {
        const int tt = tile - 2 * nth;
        kind = tt < ntv ? 2 : 3;
        const int k = tt - (kind == 3 ? ntv : 0);
        t1a = kind == 2 ? 0 : n1 - e;
        t2a = e + k * BAND_TW;
        Wd = e;
        H = min(BAND_TW, n2 - e - t2a);
    } else {
        kind = 4;
        const int c = tile - 2 * nth - 2 * ntv;
        t2a = (c & 1) ? n2 - e : 0;
        t1a = (c & 2) ? n1 - e : 0;
        H = e;
        Wd = e;
    }
    // strip coordinates: "line" across the strip, "pos" along it
    const bool horiz = kind != 2 && kind != 3;
    const int nline = horiz ? H : Wd, npos = horiz ? Wd : H;
    const int PL = nline + 2 * e, PP = npos + 2 * e;     // patch extent in line / pos
    for (int idx = threadIdx.x; idx < Ns * PL * PP; idx += blockDim.x) {
        const int i = idx / (PL * PP), rem = idx - i * PL * PP;
        const int pl = rem / PP, pp = rem - pl * PP;
        const int pr = horiz ? pl : pp, pc = horiz ? pp : pl;
        const int q2 = (t2a - e + pr) & (n2 - 1), q1 = (t1a - e + pc) & (n1 - 1);
        sm[idx] = p[(((size_t)l * Ns + i) * n2 + q2) * n1 + q1];
    }
    double2* Ds = sm + band_patch_elems(g);      // tap tables of the e lines (edge tiles)
    if (kind < 4) {
        const int per = Ns * tab;
        for (int idx = threadIdx.x; idx < e * per; idx += blockDim.x) {
            const int k = idx / per, rem = idx - k * per;
            int c2 = r - 1, c1 = r - 1;
            if (kind == 0) c2 = k;
            else if (kind == 1) c2 = r + k;
            else if (kind == 2) c1 = k;
            else c1 = r + k;
            Ds[idx] = D[((((size_t)l * nc + c2) * nc + c1) * Ns + ip) * (size_t)per + rem];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const size_t ob = ((size_t)l * Ns + ip) * g.nband;
    if (kind < 4) {
        if (wave >= nline) return;
        const int ln = wave;
        const double2* Dl = Ds + (size_t)ln * Ns * tab;   // same address in every lane: broadcast reads
        const int pos = min(lane, npos - 1);
        double2 s = cmk(0.0, 0.0);
        for (int i = 0; i < Ns; ++i) {
            const double2* Di = Dl + (size_t)i * tab;
            const double2* Pi = sm + (size_t)i * PL * PP + ln * PP + pos;
            for (int dl = 0; dl < nc; ++dl) {
                const double2* Pr = Pi + dl * PP;
#pragma unroll
                for (int dp = 0; dp < NC; ++dp) {
                    // table index [d2][d1]: (dl, dp) = (d2, d1) horizontally, (d1, d2) vertically
                    const int ti = horiz ? dl * nc + dp : dp * nc + dl;
                    s = cfma(Di[ti], Pr[dp], s);
                }
            }
        }
        if (lane < npos) {
            const int t2 = horiz ? t2a + ln : t2a + lane, t1 = horiz ? t1a + lane : t1a + ln;
            corr[ob + band_index(g, t2, t1)] = s;
        }
    } else {
        if (wave != 0) return;
        const int px = min(lane, e * e - 1);
        const int rr = px / e, cc = px - rr * e;
        const int t2 = t2a + rr, t1 = t1a + cc;
        const int c2 = band_class(t2, n2, r), c1 = band_class(t1, n1, r);
        const double2* Dl = D + ((((size_t)l * nc + c2) * nc + c1) * Ns + ip) * (size_t)Ns * tab;
        double2 s = cmk(0.0, 0.0);
        for (int i = 0; i < Ns; ++i)
            for (int d2 = 0; d2 < nc; ++d2)
                for (int d1 = 0; d1 < nc; ++d1)
                    s = cfma(Dl[((size_t)i * nc + d2) * nc + d1],
                             sm[(size_t)i * PL * PP + (rr + d2) * PP + cc + d1], s);
        if (lane < e * e) corr[ob + band_index(g, t2, t1)] = s;
    }
}

// ---------------------------------------------------------------------------
// Gram G_l = H_l^H H_l.  With z_d[q] = conj(x_i[q]) x_i'[(q + d) mod n],
//   G[(i,b),(i',b+d)] = C[d] - sum_{q2 in E(b2)} Row_d[q2] - sum_{q1 in E(b1)} Col_d[q1]
//                       + sum_{q2 in E(b2), q1 in E(b1)} z_d[q2][q1]
// where C[d] = sum_q z_d[q] (circular correlation, evaluated in the image
// domain as sum_nu conj(u_i) u_i' e^{-2 pi i d.nu/n}), E(b) = [0,b) U [b+n-r+1, n)
// the r-1 coordinates a valid anchor window misses, and Row/Col the sums of
// z_d along the band rows/columns.  Pairs i <= i' only (Hermitian).
// ---------------------------------------------------------------------------
// Per-column partials: part[x][l][pair][d2][d1]
__global__ void k_gram_col(Geo g, const double2* __restrict__ h1, const double2* __restrict__ tw2,
                           const double2* __restrict__ tw1, double2* __restrict__ part) {
    extern __shared__ double2 sm[];
    const int n1 = g.n1, n2 = g.n2, B = g.B, Ns = g.Ns, nc = g.nc, e = g.e;
    const int x1 = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    double2* U = sm;               // [B][n2]
    double2* TW2 = U + B * n2;     // [n2]
    for (int k = tid; k < n2; k += nt) TW2[k] = tw2[k];
    for (int idx = tid; idx < B * n2; idx += nt) {
        const int b = idx / n2, j = idx - b * n2;
        U[idx] = cscale(h1[((size_t)b * n1 + x1) * n2 + j], sgn_pow(j));
    }
    fft_batch_lds(U, n2, g.logn2, B, n2, TW2, true);
    const double isq2 = 1.0 / sqrt((double)n2);
    for (int idx = tid; idx < B * n2; idx += nt) {
        const int n = idx % n2;
        U[idx] = cscale(U[idx], isq2 * sgn_pow(n));
    }
    __syncthreads();
    const int nu1 = x1 - n1 / 2;
    const int nT = g.L * g.npairs * nc;
    for (int idx = tid; idx < nT; idx += nt) {
        const int d2 = idx % nc, lp = idx / nc, pair = lp % g.npairs, l = lp / g.npairs;
        int i = 0, rem = pair;
        while (rem >= Ns - i) { rem -= Ns - i; ++i; }
        const int ip = i + rem;
        const double2* ui = U + (l * Ns + i) * n2;
        const double2* uj = U + (l * Ns + ip) * n2;
        double2 t = cmk(0.0, 0.0);
        for (int n = 0; n < n2; ++n) {
            const int ph = ((d2 - e) * (n - n2 / 2)) & (n2 - 1);
            t = cfma(cconjmul(ui[n], uj[n]), TW2[ph], t);
        }
        double2* out = part + (((size_t)x1 * g.L + l) * g.npairs + pair) * nc * nc + (size_t)d2 * nc;
        for (int d1 = 0; d1 < nc; ++d1) {
            const int ph = ((d1 - e) * nu1) & (n1 - 1);
            out[d1] = cmul(t, tw1[ph]);
        }
    }
}

// C[l][pair][d] = sum_x part[x][l][pair][d] (fixed order)
__global__ void k_gram_reduce(Geo g, const double2* __restrict__ part, double2* __restrict__ C) {
    const int per = g.L * g.npairs * g.nc * g.nc;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per) return;
    double2 s = cmk(0.0, 0.0);
    for (int x = 0; x < g.n1; ++x) s = cadd(s, part[(size_t)x * per + idx]);
    C[idx] = s;
}

// Row/column sums of z_d on the band and the band corner values.
//   rows[l][pair][d][qi]      qi < 2e (band row qi)
//   cols[l][pair][d][qi]
//   cor [l][pair][d][qi2][qi1]
__global__ void k_gram_band(Geo g, const double2* __restrict__ x, double2* __restrict__ rows,
                            double2* __restrict__ cols, double2* __restrict__ cor) {
    const int n1 = g.n1, n2 = g.n2, Ns = g.Ns, nc = g.nc, e = g.e, e2 = 2 * g.e;
    const long nld = (long)g.L * g.npairs * nc * nc;
    const long n_rows = nld * e2, n_cor = nld * e2 * e2;
    const long total = 2 * n_rows + n_cor;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        int kind;  // 0 rows, 1 cols, 2 corners
        long t;
        if (idx < n_rows) { kind = 0; t = idx; }
        else if (idx < 2 * n_rows) { kind = 1; t = idx - n_rows; }
        else { kind = 2; t = idx - 2 * n_rows; }
        int qa = 0, qb = 0;
        if (kind == 2) { qb = t % e2; t /= e2; qa = t % e2; t /= e2; }
        else { qa = t % e2; t /= e2; }
        const int d1 = t % nc; t /= nc;
        const int d2 = t % nc; t /= nc;
        const int pair = t % g.npairs; t /= g.npairs;
        const int l = (int)t;
        int i = 0, rem = pair;
        while (rem >= Ns - i) { rem -= Ns - i; ++i; }
        const int ip = i + rem;
        const double2* xi = x + ((size_t)l * Ns + i) * n2 * n1;
        const double2* xj = x + ((size_t)l * Ns + ip) * n2 * n1;
        const int dd2 = d2 - e, dd1 = d1 - e;
        const size_t o = (((size_t)l * g.npairs + pair) * nc + d2) * nc + d1;
        if (kind == 0) {
            const int q2 = qa < e ? qa : n2 - e2 + qa;
            const double2* a = xi + (size_t)q2 * n1;
            const double2* bb = xj + (size_t)((q2 + dd2) & (n2 - 1)) * n1;
            double2 s = cmk(0.0, 0.0);
            for (int q1 = 0; q1 < n1; ++q1) s = cfma(cconj(a[q1]), bb[(q1 + dd1) & (n1 - 1)], s);
            rows[o * e2 + qa] = s;
        } else if (kind == 1) {
            const int q1 = qa < e ? qa : n1 - e2 + qa;
            double2 s = cmk(0.0, 0.0);
            for (int q2 = 0; q2 < n2; ++q2)
                s = cfma(cconj(xi[(size_t)q2 * n1 + q1]),
                         xj[(size_t)((q2 + dd2) & (n2 - 1)) * n1 + ((q1 + dd1) & (n1 - 1))], s);
            cols[o * e2 + qa] = s;
        } else {
            const int q2 = qa < e ? qa : n2 - e2 + qa;
            const int q1 = qb < e ? qb : n1 - e2 + qb;
            cor[(o * e2 + qa) * e2 + qb] =
                cconjmul(xi[(size_t)q2 * n1 + q1],
                         xj[(size_t)((q2 + dd2) & (n2 - 1)) * n1 + ((q1 + dd1) & (n1 - 1))]);
        }
    }
}

// G[l][row][col] for row <= col (mirrored as the conjugate).
__global__ void k_gram_assemble(Geo g, const double2* __restrict__ C, const double2* __restrict__ rows,
                                const double2* __restrict__ cols, const double2* __restrict__ cor,
                                double2* __restrict__ G) {
    const int K = g.K, r = g.r, Ns = g.Ns, nc = g.nc, e = g.e, e2 = 2 * g.e;
    const long total = (long)g.L * K * K;
    const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int l = (int)(idx / ((long)K * K));
    const int rc = (int)(idx - (long)l * K * K);
    const int row = rc / K, col = rc - row * K;
    if (row > col) return;
    const int rr2 = r * r;
    const int i = row / rr2, b2 = (row % rr2) / r, b1 = row % r;
    const int ip = col / rr2, c2 = (col % rr2) / r, c1 = col % r;
    const int pair = i * Ns - (i * (i - 1)) / 2 + (ip - i);
    const int d2 = c2 - b2 + e, d1 = c1 - b1 + e;
    const size_t o = (((size_t)l * g.npairs + pair) * nc + d2) * nc + d1;
    double2 v = C[o];
    // band indices missed by the anchor window: [0, b) and [e + b, 2e)
    for (int q = 0; q < e2; ++q) {
        const bool m2 = (q < b2) || (q >= e + b2);
        const bool m1 = (q < b1) || (q >= e + b1);
        if (m2) v = csub(v, rows[o * e2 + q]);
        if (m1) v = csub(v, cols[o * e2 + q]);
    }
    for (int qa = 0; qa < e2; ++qa) {
        if (!((qa < b2) || (qa >= e + b2))) continue;
        for (int qb = 0; qb < e2; ++qb) {
            if (!((qb < b1) || (qb >= e + b1))) continue;
            v = cadd(v, cor[(o * e2 + qa) * e2 + qb]);
        }
    }
    double2* Gl = G + (size_t)l * K * K;
    if (row == col) v.y = 0.0;
    Gl[(size_t)row * K + col] = v;
    if (row != col) Gl[(size_t)col * K + row] = cconj(v);
}

// ---------------------------------------------------------------------------
// CG vector kernels (fixed grid, grid-stride, per-block FP64 partials).
// ---------------------------------------------------------------------------
// r = b - q; partial sum |r|^2
__global__ void k_cg_init(long n, const double2* __restrict__ b, const double2* __restrict__ q,
                          double2* __restrict__ r, double* __restrict__ pr_part) {
    __shared__ double red[16];
    double s = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const double2 v = csub(b[k], q[k]);
        r[k] = v;
        s += cabs2(v);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) pr_part[blockIdx.x] = s;
}

// alpha = rr / Re<p, q>; x += alpha p; r -= alpha q; partial |r|^2.
// rr == 0 (exact solution reached) leaves x, r unchanged; a non-finite or
// non-positive curvature sets flags[0].
__global__ void k_cg_update(long n, double2* __restrict__ x, const double2* __restrict__ p,
                            double2* __restrict__ r, const double2* __restrict__ q,
                            const double* __restrict__ pr_cur, int npr, const double* __restrict__ pq_part,
                            int npq, double* __restrict__ pr_next, int* __restrict__ flags) {
    __shared__ double red[16];
    const double rr = sum_partials(pr_cur, npr, red);
    const double pq = sum_partials(pq_part, npq, red);
    double alpha = 0.0;
    if (rr > 0.0) {
        alpha = rr / pq;
        if (!(pq > 0.0) || !isfinite(alpha)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) flags[0] = 1;
            alpha = 0.0;
        }
    }
    double s = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        x[k] = cadd(x[k], cscale(p[k], alpha));
        const double2 v = csub(r[k], cscale(q[k], alpha));
        r[k] = v;
        s += cabs2(v);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) pr_next[blockIdx.x] = s;
}

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

// Coil maps c64 [L][Nc][n2][n1] -> plan layout [L][Nc][n1][n2] (x-major columns).
__global__ void k_transpose_coils(int n1, int n2, long nimg, const float2* __restrict__ S,
                                  float2* __restrict__ ST) {
    const long total = nimg * n1 * n2;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long img = k / ((long)n1 * n2);
        const int rem = (int)(k - img * n1 * n2);
        const int x = rem / n2, y = rem - x * n2;
        ST[k] = S[img * n1 * n2 + (long)y * n1 + x];
    }
}

// eps_l = mult * sigma_l for the current IRLS step (device-side schedule).
__global__ void k_eps(int L, const double* __restrict__ sigma, double mult, double* __restrict__ eps) {
    const int l = threadIdx.x;
    if (l < L) eps[l] = mult * sigma[l];
}
