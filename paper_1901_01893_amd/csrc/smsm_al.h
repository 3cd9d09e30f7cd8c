// Augmented-Lagrangian solve of Eq. 10 (Theory, "SMS MUSSELS", the
// paragraph after Eq. 10; Methods, "Reconstruction"), the solver the paper
// itself uses: the split Z_l = H_l(x_l) with scaled duals U_l, alternating
//
//   x   <- (A^H A + (beta/2) c) x = A^H y + (beta/2) sum_l H_l^H(Z_l - U_l)   (CG)
//   Z_l <- SVT_tau(M_l),  M_l = H_l(x_l) + U_l,  tau = lambda / beta
//   U_l <- M_l - Z_l
//
// (c = H^H H, the number of valid patches holding a sample).  The
// singular-value thresholding is taken as a matrix function of the K x K
// Gram, never as an SVD of the P x K matrix M:
//
//   SVT_tau(M) = M F,   F = f(M^H M),   f(s^2) = max(1 - tau / s, 0),
//
// and F is formed on the FP64 matrix cores without an eigendecomposition:
//   S  = sign(G - tau^2 I)            scaled Newton-Schulz sign iteration
//   Pr = (I + S) / 2                  projector on the singular values above tau
//   Gt = Herm(G Pr) + tau^2 (I - Pr)  equal to G there, tau^2 elsewhere
//   F  = Pr - tau Herm(Pr Gt^(-1/2))  Gt^(-1/2) by the coupled iteration of the
//                                     IRLS weights (spectrum in [tau^2, |G|])
// which equals f(G) exactly once S has converged: on singular values above
// tau, 1 - tau/s; below, 0.  Singular values within the sign iteration's
// resolution of tau are the only ones it may misplace, and there f is close
// to zero on both sides.
//
// The duals are stored [L][K][NPP] (patch index contiguous, zero beyond NP)
// so that the Gram, the dual update and the adjoint gather all read them
// along patches; M is never stored: M[p][k] = x_l[i][p2 + b2][p1 + b1] +
// U_l[k][p] with k = (i r + b2) r + b1 and p = p2 P1 + p1 (rows of H_l are
// the valid anchors p2-major, as in Eq. 8-9).
#pragma once
#include "smsm_dense.h"

struct AlGeo {
    int n1, n2, L, Ns, r, K, KP;   // K = Ns r^2, KP = K rounded up to 16
    int P1, P2, NP, NPP;           // anchors per axis, their count, NP rounded up to AL_PT
    int KB;                        // 64-wide column blocks of K
};

#define AL_BK 64    // Gram output block edge and dual-update row block
#define AL_SL 16    // Gram: patches per staged slab
#define AL_PT 64    // dual update: patches per tile
#define AL_STR 65   // shared-memory row stride (complex entries): 16-byte rows land 4 banks apart

// number of valid r-wide windows along an axis of n samples holding sample t
SMSM_HD inline int al_cnt(int t, int n, int r) {
    int c = t + 1 < r ? t + 1 : r;
    const int d = n - t < n - r + 1 ? n - t : n - r + 1;
    return c < d ? c : d;
}

// Offset of the x sample of column k at anchor 0 (k < K), or -1 (k >= K).
SMSM_DEV int al_col_off(const AlGeo& a, int k) {
    if (k >= a.K) return -1;
    const int r2 = a.r * a.r;
    const int i = k / r2, rem = k - i * r2, b2 = rem / a.r, b1 = rem - b2 * a.r;
    return (i * a.n2 + b2) * a.n1 + b1;
}

// G partials: block pair (I <= J) of 64 x 64 outputs of sum_p conj(M[p][a]) M[p][b]
// over one chunk of `chunk` patches.  grid (KB (KB + 1) / 2, nchunk, L), block 256:
// wave w computes the 32 x 32 quarter (w >> 1, w & 1) as 2 x 2 tiles of
// v_mfma_f64_16x16x4f64 (three real products per complex step, as in k_zgemm);
// slabs of 16 patches of both column blocks (the same one twice on the
// diagonal) are staged in shared memory, the
// next slab's loads in flight during the current slab's products.
// part[l][chunk][pair][64][64] (tiles outside K written as zero).
__global__ void __launch_bounds__(256, 2) k_al_gram(AlGeo a, const double2* __restrict__ x,
                                                 const double2* __restrict__ U, int chunk,
                                                 double2* __restrict__ part) {
    __shared__ double2 sa[AL_SL][AL_STR];
    __shared__ double2 sb[AL_SL][AL_STR];
    const int l = blockIdx.z, c = blockIdx.y, npair = gridDim.x;
    int I = 0, J = blockIdx.x;
    while (J >= a.KB - I) {
        J -= a.KB - I;
        ++I;
    }
    J += I;
    const bool diag = I == J;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wa = w >> 1, wb = w & 1;
    const double2* xl = x + (size_t)l * a.Ns * a.n2 * a.n1;
    const double2* Ul = U + (size_t)l * a.K * a.NPP;
    const int p_beg = c * chunk;
    const int p_end = min(p_beg + chunk, a.NP);
    // staging: patch pp of the slab, columns cc0 + 16 s of each block
    const int pp = tid & 15, cc0 = tid >> 4;
    int offA[4], offB[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        offA[s] = al_col_off(a, I * AL_BK + cc0 + 16 * s);
        offB[s] = al_col_off(a, J * AL_BK + cc0 + 16 * s);
    }
    double2 va[4], vb[4];
    auto load = [&](int p0) {
        const int p = p0 + pp;
        const bool ok = p < p_end;
        int po = 0;
        if (ok) {
            const int p2 = p / a.P1;
            po = p2 * a.n1 + (p - p2 * a.P1);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            va[s] = (ok && offA[s] >= 0)
                        ? cadd(xl[offA[s] + po], Ul[(size_t)(I * AL_BK + cc0 + 16 * s) * a.NPP + p])
                        : cmk(0.0, 0.0);
            vb[s] = diag ? va[s]
                         : (ok && offB[s] >= 0)
                               ? cadd(xl[offB[s] + po], Ul[(size_t)(J * AL_BK + cc0 + 16 * s) * a.NPP + p])
                               : cmk(0.0, 0.0);
        }
    };
    const int row0 = I * AL_BK + wa * 32, col0 = J * AL_BK + wb * 32;
    const bool rv[2] = {row0 < a.K, row0 + 16 < a.K};
    const bool cv[2] = {col0 < a.K, col0 + 16 < a.K};
    hd4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            t1[i][j] = hd4{0.0, 0.0, 0.0, 0.0};
            t2[i][j] = t1[i][j];
            t3[i][j] = t1[i][j];
        }
    if (p_beg < p_end) load(p_beg);
    for (int p0 = p_beg; p0 < p_end; p0 += AL_SL) {
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            sa[pp][cc0 + 16 * s] = va[s];
            sb[pp][cc0 + 16 * s] = vb[s];
        }
        __syncthreads();
        if (p0 + AL_SL < p_end) load(p0 + AL_SL);
        if (rv[0] && cv[0]) {
#pragma unroll
            for (int st = 0; st < AL_SL / 4; ++st) {
                const int q = 4 * st + (lane >> 4);
                double2 av[2], bv[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    av[t] = sa[q][wa * 32 + 16 * t + (lane & 15)];
                    bv[t] = sb[q][wb * 32 + 16 * t + (lane & 15)];
                }
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    if (!rv[i]) continue;
                    const double ar = av[i].x, ai = -av[i].y;   // conj(M[p][a])
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        if (!cv[j]) continue;
                        const double br = bv[j].x, bi = bv[j].y;
                        t1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, br, t1[i][j], 0, 0, 0);
                        t2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi - br, t2[i][j], 0, 0, 0);
                        t3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br + bi, t3[i][j], 0, 0, 0);
                    }
                }
            }
        }
    }
    double2* out = part + (((size_t)l * gridDim.y + c) * npair + blockIdx.x) * AL_BK * AL_BK;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const hd4 cr = t1[i][j] - t3[i][j], ci = t1[i][j] + t2[i][j];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wa * 32 + 16 * i + 4 * v + (lane >> 4), col = wb * 32 + 16 * j + (lane & 15);
                out[row * AL_BK + col] = cmk(cr[v], ci[v]);
            }
        }
}

// Index of block pair (I, J), I <= J, in k_al_gram's enumeration.
SMSM_DEV int al_pair(int I, int J, int KB) { return I * KB - I * (I - 1) / 2 + (J - I); }

// G_l (padded KP x KP, exactly Hermitian: the lower triangle mirrors the
// upper) from the chunk partials added in chunk order, Q_l = G_l - tau^2 I
// (identity of the K x K block) and per-block partials of ||Q_l||_F^2.
// grid (kPad, L).
__global__ void k_al_gram_sum(AlGeo a, const double2* __restrict__ part, int nchunk, double tau2,
                              double2* __restrict__ G, double2* __restrict__ Q, double* __restrict__ qpart) {
    __shared__ double red[16];
    const int l = blockIdx.y, npair = a.KB * (a.KB + 1) / 2;
    double s2 = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < a.KP * a.KP; idx += gridDim.x * blockDim.x) {
        const int i = idx / a.KP, j = idx - i * a.KP;
        double2 g = cmk(0.0, 0.0);
        if (i < a.K && j < a.K) {
            const bool up = i <= j;
            const int u = up ? i : j, v = up ? j : i;
            const int bi = u / AL_BK, bj = v / AL_BK;
            const size_t o = (size_t)al_pair(bi, bj, a.KB) * AL_BK * AL_BK + (u % AL_BK) * AL_BK + v % AL_BK;
            for (int c = 0; c < nchunk; ++c)
                g = cadd(g, part[((size_t)l * nchunk + c) * npair * AL_BK * AL_BK + o]);
            if (!up) g = cconj(g);
            if (i == j) g.y = 0.0;
        }
        const size_t o = (size_t)l * a.KP * a.KP + idx;
        G[o] = g;
        const double2 q = (i == j && i < a.K) ? cmk(g.x - tau2, 0.0) : g;
        Q[o] = q;
        s2 += cabs2(q);
    }
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) qpart[(size_t)l * gridDim.x + blockIdx.x] = s2;
}

// X_l = Q_l / ||Q_l||_F (the sign iteration's start, spectrum in [-1, 1]);
// a zero Q_l stays zero.  grid (kPad, L).
__global__ void k_al_sign_start(int KP, const double2* __restrict__ Q, const double* __restrict__ qpart, int np,
                                double2* __restrict__ X) {
    __shared__ double red[16];
    const int l = blockIdx.y;
    const double f2 = sum_partials(qpart + (size_t)l * np, np, red);
    const double ic = f2 > 0.0 ? 1.0 / sqrt(f2) : 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < KP * KP; idx += gridDim.x * blockDim.x) {
        const size_t o = (size_t)l * KP * KP + idx;
        X[o] = cscale(Q[o], ic);
    }
}

// Pr = (I + S) / 2 on the K x K block (zero padding).  grid (kPad, L).
__global__ void k_al_proj(int K, int KP, const double2* __restrict__ S, double2* __restrict__ Pr) {
    const int l = blockIdx.y;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < KP * KP; idx += gridDim.x * blockDim.x) {
        const int i = idx / KP, j = idx - i * KP;
        const size_t o = (size_t)l * KP * KP + idx;
        double2 v = cmk(0.0, 0.0);
        if (i < K && j < K) v = cmk(0.5 * (S[o].x + (i == j ? 1.0 : 0.0)), 0.5 * S[o].y);
        Pr[o] = v;
    }
}

// Gt = Herm(C) + tau^2 (I - Pr) with C = G Pr, into Y (the coupled
// iteration's start buffer), and per-block partials of ||Gt||_F^2.
// grid (kPad, L).
__global__ void k_al_gtilde(int K, int KP, const double2* __restrict__ C, const double2* __restrict__ Pr,
                            double tau2, double2* __restrict__ Y, double* __restrict__ part) {
    __shared__ double red[16];
    const int l = blockIdx.y;
    const size_t base = (size_t)l * KP * KP;
    double s2 = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < KP * KP; idx += gridDim.x * blockDim.x) {
        const int i = idx / KP, j = idx - i * KP;
        double2 v = cmk(0.0, 0.0);
        if (i < K && j < K) {
            const double2 u = C[base + idx], t = C[base + (size_t)j * KP + i], p = Pr[base + idx];
            v = cmk(0.5 * (u.x + t.x) + tau2 * ((i == j ? 1.0 : 0.0) - p.x), 0.5 * (u.y - t.y) - tau2 * p.y);
            if (i == j) v.y = 0.0;
        }
        Y[base + idx] = v;
        s2 += cabs2(v);
    }
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) part[(size_t)l * gridDim.x + blockIdx.x] = s2;
}

// Wp_l = wscale_l Z_l with Z_l from the buffer the coupled iteration last
// wrote; flags[1] = 1 when a slice did not meet the tolerance.  grid (kPad, L).
__global__ void k_al_pick(int K, int KP, const double2* __restrict__ Z0, const double2* __restrict__ Z1,
                          const int* __restrict__ last, const int* __restrict__ conv,
                          const double* __restrict__ wscale, double2* __restrict__ Wp, int* __restrict__ flags) {
    const int l = blockIdx.y;
    if (blockIdx.x == 0 && threadIdx.x == 0 && !conv[l]) flags[1] = 1;
    const double2* Z = last[l] ? Z1 : Z0;
    const double ws = wscale[l];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < KP * KP; idx += gridDim.x * blockDim.x) {
        const size_t o = (size_t)l * KP * KP + idx;
        Wp[o] = cscale(Z[o], ws);
    }
}

// F = Pr - tau Herm(C) with C = Pr Wp.  grid (kPad, L).
__global__ void k_al_f(int K, int KP, const double2* __restrict__ C, const double2* __restrict__ Pr, double tau,
                       double2* __restrict__ F) {
    const int l = blockIdx.y;
    const size_t base = (size_t)l * KP * KP;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < KP * KP; idx += gridDim.x * blockDim.x) {
        const int i = idx / KP, j = idx - i * KP;
        double2 v = cmk(0.0, 0.0);
        if (i < K && j < K) {
            const double2 u = C[base + idx], t = C[base + (size_t)j * KP + i], p = Pr[base + idx];
            v = cmk(p.x - tau * 0.5 * (u.x + t.x), p.y - tau * 0.5 * (u.y - t.y));
            if (i == j) v.y = 0.0;
        }
        F[base + idx] = v;
    }
}

// Dual update U_out = M - M F (M = H(x) + U_in), written [k][p].  The product
// is taken transposed, T^T[k][p] = sum_j F[j][k] M[p][j], so that the
// matrix cores' output tile runs along patches.  grid (NPP / AL_PT * KBU, 1, L)
// with KBU = ceil(K / (16 NW)), block 64 NW: workgroup (patch tile, 16 NW rows
// of k), wave w the 16 rows 16 w of the block against the tile's 64 patches
// (4 tiles of v_mfma_f64_16x16x4f64); chunks of 16 j of M^T and F staged in
// shared memory, the next chunk's loads in flight during the current chunk's
// products.  More rows per workgroup stage each patch tile's M^T fewer times.
template <int NW>
__global__ void __launch_bounds__(64 * NW, 8 / NW) k_al_update(AlGeo a, const double2* __restrict__ x,
                                                               const double2* __restrict__ Uin,
                                                               const double2* __restrict__ F,
                                                               double2* __restrict__ Uout) {
    constexpr int NT = 64 * NW, KR = 16 * NW;
    constexpr int SM_IT = 16 * AL_PT / NT, SF_IT = 16 * KR / NT;   // staged entries per thread
    __shared__ double2 sm[16][AL_STR];      // M^T chunk [j][p]
    __shared__ double2 sf[16][KR + 1];      // F chunk [j][k]
    const int l = blockIdx.z;
    const int kbu = (a.K + KR - 1) / KR;
    const int tile = blockIdx.x / kbu, kb = blockIdx.x - tile * kbu;
    const int p0 = tile * AL_PT, k0 = kb * KR;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double2* xl = x + (size_t)l * a.Ns * a.n2 * a.n1;
    const double2* Ul = Uin + (size_t)l * a.K * a.NPP;
    const double2* Fl = F + (size_t)l * a.KP * a.KP;
    // staging of M^T: entry e = tid + s NT -> patch e & 63, row e >> 6
    int po[SM_IT];
    bool pok[SM_IT];
#pragma unroll
    for (int s = 0; s < SM_IT; ++s) {
        const int p = p0 + ((tid + s * NT) & 63);
        pok[s] = p < a.NP;
        const int p2 = pok[s] ? p / a.P1 : 0;
        po[s] = pok[s] ? p2 * a.n1 + (p - p2 * a.P1) : 0;
    }
    double2 vm[SM_IT], vf[SF_IT];
    auto load = [&](int j0) {
#pragma unroll
        for (int s = 0; s < SM_IT; ++s) {
            const int e = tid + s * NT;
            const int j = j0 + (e >> 6);
            const int off = al_col_off(a, j);
            vm[s] = (pok[s] && off >= 0) ? cadd(xl[off + po[s]], Ul[(size_t)j * a.NPP + p0 + (e & 63)])
                                         : cmk(0.0, 0.0);
        }
#pragma unroll
        for (int s = 0; s < SF_IT; ++s) {
            const int e = tid + s * NT;
            const int j = j0 + e / KR, kk = k0 + e % KR;
            vf[s] = (kk < a.K && j < a.K) ? Fl[(size_t)j * a.KP + kk] : cmk(0.0, 0.0);
        }
    };
    const bool wok = k0 + 16 * w < a.K;
    hd4 t1[4], t2[4], t3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        t1[t] = hd4{0.0, 0.0, 0.0, 0.0};
        t2[t] = t1[t];
        t3[t] = t1[t];
    }
    load(0);
    for (int j0 = 0; j0 < a.K; j0 += 16) {
        __syncthreads();
#pragma unroll
        for (int s = 0; s < SM_IT; ++s) {
            const int e = tid + s * NT;
            sm[e >> 6][e & 63] = vm[s];
        }
#pragma unroll
        for (int s = 0; s < SF_IT; ++s) {
            const int e = tid + s * NT;
            sf[e / KR][e % KR] = vf[s];
        }
        __syncthreads();
        if (j0 + 16 < a.K) load(j0 + 16);
        if (wok) {
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int q = 4 * st + (lane >> 4);
                const double2 av = sf[q][16 * w + (lane & 15)];   // A[k][j] = F[j][k]
                double2 bv[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) bv[t] = sm[q][16 * t + (lane & 15)];   // B[j][p] = M[p][j]
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    t1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x + av.y, bv[t].x, t1[t], 0, 0, 0);
                    t2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv[t].y - bv[t].x, t2[t], 0, 0, 0);
                    t3[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv[t].x + bv[t].y, t3[t], 0, 0, 0);
                }
            }
        }
    }
    if (!wok) return;
    double2* Uo = Uout + (size_t)l * a.K * a.NPP;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const hd4 cr = t1[t] - t3[t], ci = t1[t] + t2[t];
        const int pc = p0 + 16 * t + (lane & 15);
        int pco = 0;
        const bool ok = pc < a.NP;
        if (ok) {
            const int p2 = pc / a.P1;
            pco = p2 * a.n1 + (pc - p2 * a.P1);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = k0 + 16 * w + 4 * v + (lane >> 4);
            if (k >= a.K) continue;
            double2 u = cmk(0.0, 0.0);
            if (ok) {
                const double2 m = cadd(xl[al_col_off(a, k) + pco], Ul[(size_t)k * a.NPP + pc]);
                u = cmk(m.x - cr[v], m.y - ci[v]);
            }
            Uo[(size_t)k * a.NPP + pc] = u;
        }
    }
}

// hu = H^H(U) per sample (the valid anchors' entries summed in (b2, b1)
// order), then hzu = c x + hu_old - 2 hu, which is H^H(Z - U) for the split
// Z = M - U of the update just made (M = H(x) + U_old).  One thread per
// sample of [L][Ns][n2][n1].
__global__ void k_al_gather(AlGeo a, const double2* __restrict__ x, const double2* __restrict__ U,
                            double2* __restrict__ hu, double2* __restrict__ hzu) {
    const long n = (long)a.L * a.Ns * a.n2 * a.n1;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
        const int q1 = (int)(idx % a.n1);
        long t = idx / a.n1;
        const int q2 = (int)(t % a.n2);
        t /= a.n2;
        const int i = (int)(t % a.Ns), l = (int)(t / a.Ns);
        const double2* Ul = U + (size_t)l * a.K * a.NPP;
        double2 s = cmk(0.0, 0.0);
        for (int b2 = 0; b2 < a.r; ++b2) {
            const int p2 = q2 - b2;
            if (p2 < 0 || p2 >= a.P2) continue;
            for (int b1 = 0; b1 < a.r; ++b1) {
                const int p1 = q1 - b1;
                if (p1 < 0 || p1 >= a.P1) continue;
                s = cadd(s, Ul[(size_t)((i * a.r + b2) * a.r + b1) * a.NPP + p2 * a.P1 + p1]);
            }
        }
        const double c = (double)(al_cnt(q2, a.n2, a.r) * al_cnt(q1, a.n1, a.r));
        const double2 h = hu[idx], xv = x[idx];
        hzu[idx] = cmk(c * xv.x + h.x - 2.0 * s.x, c * xv.y + h.y - 2.0 * s.y);
        hu[idx] = s;
    }
}

// Start of the splitting: hzu = c x (= H^H H x, the split Z = H(x) with
// U = 0), hu = 0.
__global__ void k_al_init(AlGeo a, const double2* __restrict__ x, double2* __restrict__ hu,
                          double2* __restrict__ hzu) {
    const long n = (long)a.L * a.Ns * a.n2 * a.n1;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
        const int q1 = (int)(idx % a.n1), q2 = (int)((idx / a.n1) % a.n2);
        const double c = (double)(al_cnt(q2, a.n2, a.r) * al_cnt(q1, a.n1, a.r));
        hzu[idx] = cscale(x[idx], c);
        hu[idx] = cmk(0.0, 0.0);
    }
}

// out += f c v (the x-step's diagonal term, f = beta / 2).
__global__ void k_al_diag(AlGeo a, const double2* __restrict__ v, double f, double2* __restrict__ out) {
    const long n = (long)a.L * a.Ns * a.n2 * a.n1;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
        const int q1 = (int)(idx % a.n1), q2 = (int)((idx / a.n1) % a.n2);
        const double c = f * (double)(al_cnt(q2, a.n2, a.r) * al_cnt(q1, a.n1, a.r));
        out[idx] = cadd(out[idx], cscale(v[idx], c));
    }
}
