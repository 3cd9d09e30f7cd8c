// The Hankel Gram G_l = H_l(x_l)^H H_l(x_l) (Eq. 8-9) as a GEMM over the patch
// anchors on the BF16 matrix cores: the mixed-precision form of the Gram.
// Every entry x = a + i b of H is split into three BF16 parts per real
// component (a = a0 + a1 + a2, each part the round to nearest of what the
// previous ones left, to about 2^-24 |a|), and each real product is formed
// from the six part products a_i b_j with i + j <= 2 (the cross terms
// compensate the rounding of the leading parts; the three smallest are
// dropped), accumulated in FP32 over a chunk of GB_CH patches and in FP64
// across chunks:
//   Re G[a][b] = sum_p (Re M[p][a] Re M[p][b] + Im M[p][a] Im M[p][b])
//   Im G[a][b] = sum_p (Re M[p][a] Im M[p][b] - Im M[p][a] Re M[p][b])
// with M[p][k] = x_l[i][p2 + b2][p1 + b1], k = (i r + b2) r + b1.
// MFMA operand layout (v_mfma_f32_16x16x32_bf16): lane l holds
// A[m = l % 16][k = 8 (l / 16) + j] and B[k = 8 (l / 16) + j][n = l % 16], so both
// operands are eight consecutive patches of one column; a slab of 32 patches
// of the two column blocks is staged in shared memory as
// [part][re, im][column][patch] (column stride GB_CST BF16, which puts the 16
// columns of a fragment read on distinct banks).
#pragma once
#include "smsm_al.h"
#include "smsm_cnn_mfma.h"

#define GB_SL 32     // patches per staged slab (one MFMA K step)
#define GB_CH 2048   // patches per chunk (FP32 accumulation)
#define GB_CST 40    // BF16 per staged column (32 patches + 8 spread)

// Block pair (I <= J) of 64 x 64 outputs over one chunk of patches.
// grid (KB (KB + 1) / 2, nchunk, L), block 256: wave w computes the 32 x 32
// quarter (w >> 1, w & 1) as 2 x 2 tiles.  part[l][chunk][pair][64][64] (FP64;
// tiles outside K written as zero).
__global__ void __launch_bounds__(256, 2) k_gram_bf16(AlGeo a, const double2* __restrict__ x,
                                                      double2* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) unsigned short sm[2][3][2][64 * GB_CST];   // [block][part][re/im]
    const int l = blockIdx.z, c = blockIdx.y, npair = gridDim.x;
    int I = 0, J = blockIdx.x;
    while (J >= a.KB - I) {
        J -= a.KB - I;
        ++I;
    }
    J += I;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wa = w >> 1, wb = w & 1;
    const int g = lane >> 4, l16 = lane & 15;
    const double2* xl = x + (size_t)l * a.Ns * a.n2 * a.n1;
    const int p_beg = c * GB_CH;
    const int p_end = min(p_beg + GB_CH, a.NP);
    const int row0 = I * 64 + wa * 32, col0 = J * 64 + wb * 32;
    const bool rv[2] = {row0 < a.K, row0 + 16 < a.K};
    const bool cv[2] = {col0 < a.K, col0 + 16 < a.K};
    cm_f32x4 accR[2][2], accI[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            accR[i][j] = cm_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            accI[i][j] = accR[i][j];
        }
    // staging tasks (block, column, 8-patch group): two per thread
    int soff[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int t = tid + 256 * u, blk = t >> 8, col = (t >> 2) & 63;
        soff[u] = al_col_off(a, (blk ? J : I) * 64 + col);
    }
    for (int p0 = p_beg; p0 < p_end; p0 += GB_SL) {
        __syncthreads();                                // the previous slab's fragments are read
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = tid + 256 * u, blk = t >> 8, col = (t >> 2) & 63, grp = t & 3;
            unsigned pk[3][2][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double va[2][2];                        // [pixel of the pair][re, im]
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int p = p0 + 8 * grp + 2 * q + h;
                    double2 v = cmk(0.0, 0.0);
                    if (soff[u] >= 0 && p < p_end) {
                        const int p2 = p / a.P1;
                        v = xl[soff[u] + p2 * a.n1 + (p - p2 * a.P1)];
                    }
                    va[h][0] = v.x;
                    va[h][1] = v.y;
                }
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    double r0 = va[0][ri], r1 = va[1][ri];
#pragma unroll
                    for (int pt = 0; pt < 3; ++pt) {   // parts: round to nearest of the remainder
                        const unsigned h0 = cm_bf16_bits((float)r0), h1 = cm_bf16_bits((float)r1);
                        pk[pt][ri][q] = h0 | (h1 << 16);
                        r0 -= (double)__uint_as_float(h0 << 16);
                        r1 -= (double)__uint_as_float(h1 << 16);
                    }
                }
            }
#pragma unroll
            for (int pt = 0; pt < 3; ++pt)
#pragma unroll
                for (int ri = 0; ri < 2; ++ri)
                    *reinterpret_cast<uint4*>(&sm[blk][pt][ri][col * GB_CST + 8 * grp]) =
                        make_uint4(pk[pt][ri][0], pk[pt][ri][1], pk[pt][ri][2], pk[pt][ri][3]);
        }
        __syncthreads();
        if (!(rv[0] && cv[0])) continue;
        // the wave's fragments: rows (block I) and columns (block J), three parts, re and im
        cm_bf16x8 fa[2][3][2], fb[2][3][2];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int pt = 0; pt < 3; ++pt)
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    fa[t][pt][ri] = *reinterpret_cast<const cm_bf16x8*>(
                        &sm[0][pt][ri][(wa * 32 + 16 * t + l16) * GB_CST + 8 * g]);
                    fb[t][pt][ri] = *reinterpret_cast<const cm_bf16x8*>(
                        &sm[1][pt][ri][(wb * 32 + 16 * t + l16) * GB_CST + 8 * g]);
                }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            if (!rv[i]) continue;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (!cv[j]) continue;
#pragma unroll
                for (int pa = 0; pa < 3; ++pa)
#pragma unroll
                    for (int pb = 0; pb + pa < 3; ++pb) {
                        const cm_bf16x8 ar = fa[i][pa][0], ai = fa[i][pa][1];
                        const cm_bf16x8 br = fb[j][pb][0], bi = fb[j][pb][1];
                        const cm_bf16x8 nai = __builtin_bit_cast(
                            cm_bf16x8, __builtin_bit_cast(uint4, ai) ^ make_uint4(0x80008000u, 0x80008000u,
                                                                                 0x80008000u, 0x80008000u));
                        accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br, accR[i][j], 0, 0, 0);
                        accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, bi, accR[i][j], 0, 0, 0);
                        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, bi, accI[i][j], 0, 0, 0);
                        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai, br, accI[i][j], 0, 0, 0);
                    }
            }
        }
    }
    double2* out = part + (((size_t)l * gridDim.y + c) * npair + blockIdx.x) * 64 * 64;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wa * 32 + 16 * i + 4 * g + v, col = wb * 32 + 16 * j + l16;
                out[row * 64 + col] = cmk((double)accR[i][j][v], (double)accI[i][j][v]);
            }
}

// G_l [K][K] (exactly Hermitian: the lower triangle mirrors the upper, a real
// diagonal) from the chunk partials added in chunk order (FP64).  grid
// (kPad, L).
__global__ void k_gram_bf16_sum(AlGeo a, const double2* __restrict__ part, int nchunk, double2* __restrict__ G) {
    const int l = blockIdx.y, npair = a.KB * (a.KB + 1) / 2;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < a.K * a.K; idx += gridDim.x * blockDim.x) {
        const int i = idx / a.K, j = idx - i * a.K;
        const bool up = i <= j;
        const int u = up ? i : j, v = up ? j : i;
        const size_t o = (size_t)al_pair(u / 64, v / 64, a.KB) * 64 * 64 + (u % 64) * 64 + v % 64;
        double2 s = cmk(0.0, 0.0);
        for (int c = 0; c < nchunk; ++c) s = cadd(s, part[((size_t)l * nchunk + c) * npair * 64 * 64 + o]);
        if (!up) s = cconj(s);
        if (i == j) s.y = 0.0;
        G[(size_t)l * a.K * a.K + idx] = s;
    }
}
