// Hankel Gram matrices G_l = H_l^H H_l of the current iterate (Eq. 8-9).
//
// With z_d[q] = conj(x_i[q]) x_i'[(q + d) mod n] (shot pair i <= i', lag d in
// [-e, e]^2, e = r-1),
//   G[(i,b),(i',b+d)] = C[d] - sum_{q2 in E(b2)} Row_d[q2] - sum_{q1 in E(b1)} Col_d[q1]
//                       + sum_{q2 in E(b2), q1 in E(b1)} z_d[q2][q1]
// where C[d] = sum_q z_d[q] is the circular correlation, E(b) = [0,b) U
// [b+n-r+1, n) the e coordinates an anchor window at offset b misses, and
// Row/Col are the sums of z_d along the band rows/columns (the 2e rows and
// columns within e of an edge).  C is evaluated in the image domain:
//   C[d] = sum_x e^{-2 pi i d1 (x-n1/2)/n1} sum_n conj(u_i[x][n]) u_i'[x][n] e^{-2 pi i d2 (n-n2/2)/n2}
// with u the centred unitary inverse DFT of x along ky (columns of the hybrid
// layout h1, already inverse-transformed along kx).  The inner sum is one
// in-wave FFT of the product per (pair, column); its 2e+1 bins around zero
// are the d2 lags.
#pragma once
#include "smsm_wavefft.h"

// Pair index of (i, i'), i <= i': i Ns - i (i - 1) / 2 + (i' - i).
SMSM_DEV void gram_pair(int pair, int Ns, int& i, int& ip) {
    int rem = pair;
    i = 0;
    while (rem >= Ns - i) {
        rem -= Ns - i;
        ++i;
    }
    ip = i + rem;
}

// Lanes of a wave split into groups of GS = 16 (4 groups; 2r-1 <= 16) or
// 32 (2 groups): lane = j + GS g.  Sum over the groups, fixed order.
SMSM_DEV int gram_gs(int nc) { return nc <= 16 ? 16 : 32; }
SMSM_DEV double2 gram_reduce_groups(double2 v, int gs) {
    if (gs == 16) v = cadd(v, lane_xor2<16>(v));
    v = cadd(v, lane_xor2<32>(v));
    return v;
}

// Q[l][pair][x][d2] = sum_n conj(u_i[x][n]) u_i'[x][n] e^{-2 pi i (d2-e)(n-n2/2)/n2}.
// One workgroup (4 waves) per column x: the 12 (L Ns) columns are inverse
// transformed into shared memory, then each wave takes pairs in turn:
// product, forward in-wave FFT, and the bins (d2 - e) mod n2, times (-1)^(d2-e).
template <int N2>
__global__ void __launch_bounds__(256)
k_gram_q(Geo g, const double2* __restrict__ h1, const double2* __restrict__ tw2, double2* __restrict__ Q) {
    using F = WaveFft<N2>;
    constexpr int R = F::R, LANES = F::LANES, G = 64 / LANES;
    extern __shared__ double2 sm[];
    const int n1 = g.n1, B = g.B, Ns = g.Ns, nc = g.nc, e = g.e, npairs = g.npairs;
    const int x = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int grp = lane / LANES;
    double2* U = sm;                 // [B][N2]
    double2* TW = sm + B * N2;       // [N2]
    for (int k = threadIdx.x; k < N2; k += blockDim.x) TW[k] = tw2[k];
    __syncthreads();
    F f;
    f.setup(TW, lane);
    const double isq = 1.0 / sqrt((double)N2);
    for (int b0 = wave * G; b0 < B; b0 += nw * G) {
        const int b = b0 + grp;
        if (b < B) {
            const double2* src = h1 + ((size_t)b * n1 + x) * N2;
            double2 v[R];
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int k = f.m + 64 * t;
                v[t] = cscale(src[k], sgn_pow(k));
            }
            f.template run<true>(v);
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int n = f.out_index(t);
                U[b * N2 + n] = cscale(v[t], isq * sgn_pow(n));
            }
        }
    }
    __syncthreads();
    const int ntask = g.L * npairs;
    for (int t0 = wave * G; t0 < ntask; t0 += nw * G) {
        const int task = t0 + grp;
        if (task < ntask) {
            const int l = task / npairs, pair = task - l * npairs;
            int i, ip;
            gram_pair(pair, Ns, i, ip);
            const double2* ui = U + (l * Ns + i) * N2;
            const double2* uj = U + (l * Ns + ip) * N2;
            double2 v[R];
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int n = f.m + 64 * t;
                v[t] = cconjmul(ui[n], uj[n]);
            }
            f.template run<false>(v);
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int k = f.out_index(t);
                const int d2 = k <= e ? k + e : k - (N2 - e);
                if (d2 >= 0 && d2 < nc && (k <= e || k >= N2 - e))
                    Q[(((size_t)l * npairs + pair) * n1 + x) * nc + d2] = cscale(v[t], sgn_pow(d2 - e));
            }
        }
    }
}

// C[l][pair][d2][d1] = sum_x Q[l][pair][x][d2] e^{-2 pi i (d1-e)(x-n1/2)/n1}.
// One wave per (l, pair, d2); lane = d1 + GS g sums the x of group g.
__global__ void __launch_bounds__(256)
k_gram_c(Geo g, const double2* __restrict__ Q, const double2* __restrict__ tw1, double2* __restrict__ C) {
    const int n1 = g.n1, nc = g.nc, e = g.e;
    const int wv = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int nwv = g.L * g.npairs * nc;
    if (wv >= nwv) return;
    const int gs = gram_gs(nc), ng = 64 / gs;
    const int lane = threadIdx.x & 63, d1 = lane & (gs - 1), qg = lane / gs;
    const int lp = wv / nc, d2 = wv - lp * nc;      // lp = l * npairs + pair
    const int xq = n1 / ng, x0 = qg * xq;
    const double2* q = Q + (size_t)lp * n1 * nc + d2;
    double2 s = cmk(0.0, 0.0);
    if (d1 < nc) {
#pragma unroll 8
        for (int x = x0; x < x0 + xq; ++x)
            s = cfma(q[(size_t)x * nc], tw1[((d1 - e) * (x - n1 / 2)) & (n1 - 1)], s);
    }
    s = gram_reduce_groups(s, gs);
    if (qg == 0 && d1 < nc) C[((size_t)lp * nc + d2) * nc + d1] = s;
}

// Band row and column sums of z_d.  One wave per (kind, l, pair, fixed lag,
// band line qa); lane = (free lag) + GS g sums the positions of group g:
//   rows[l][pair][d2][d1][qa] = sum_q1 conj(x_i[q2][q1]) x_i'[q2+d2-e][q1+d1-e],  q2 = band row qa
//   cols[l][pair][d2][d1][qa] = sum_q2 conj(x_i[q2][q1]) x_i'[q2+d2-e][q1+d1-e],  q1 = band col qa
// (rows: wave fixes d2, lanes d1; cols: wave fixes d1, lanes d2).
__global__ void __launch_bounds__(256)
k_gram_lines(Geo g, const double2* __restrict__ x, double2* __restrict__ rows, double2* __restrict__ cols) {
    const int n1 = g.n1, n2 = g.n2, Ns = g.Ns, nc = g.nc, e = g.e, e2 = 2 * g.e;
    const int per = g.L * g.npairs * nc * e2;
    const int wv = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wv >= 2 * per) return;
    const bool col = wv >= per;
    int t = col ? wv - per : wv;
    const int qa = t % e2;
    t /= e2;
    const int fixed = t % nc;
    const int lp = t / nc, l = lp / g.npairs, pair = lp - l * g.npairs;
    int i, ip;
    gram_pair(pair, Ns, i, ip);
    const int gs = gram_gs(nc), ng = 64 / gs;
    const int lane = threadIdx.x & 63, fr = lane & (gs - 1), qg = lane / gs;
    const double2* xi = x + ((size_t)l * Ns + i) * n2 * n1;
    const double2* xj = x + ((size_t)l * Ns + ip) * n2 * n1;
    double2 s = cmk(0.0, 0.0);
    if (fr < nc) {
        if (!col) {
            const int q2 = qa < e ? qa : n2 - e2 + qa;
            const double2* a = xi + (size_t)q2 * n1;
            const double2* b = xj + (size_t)((q2 + fixed - e) & (n2 - 1)) * n1;
            const int len = n1 / ng, q0 = qg * len;
#pragma unroll 8
            for (int q1 = q0; q1 < q0 + len; ++q1) s = cfma(cconj(a[q1]), b[(q1 + fr - e) & (n1 - 1)], s);
        } else {
            const int q1 = qa < e ? qa : n1 - e2 + qa;
            const int c1 = (q1 + fixed - e) & (n1 - 1);
            const int len = n2 / ng, q0 = qg * len;
#pragma unroll 8
            for (int q2 = q0; q2 < q0 + len; ++q2)
                s = cfma(cconj(xi[(size_t)q2 * n1 + q1]), xj[(size_t)((q2 + fr - e) & (n2 - 1)) * n1 + c1], s);
        }
    }
    s = gram_reduce_groups(s, gs);
    if (qg == 0 && fr < nc) {
        const int d2 = col ? fr : fixed, d1 = col ? fixed : fr;
        const size_t o = (((size_t)lp * nc + d2) * nc + d1) * e2 + qa;
        (col ? cols : rows)[o] = s;
    }
}

// Corner values cor[l][pair][d2][d1][qa][qb] = z_d[band row qa][band col qb].
__global__ void k_gram_corners(Geo g, const double2* __restrict__ x, double2* __restrict__ cor) {
    const int n1 = g.n1, n2 = g.n2, Ns = g.Ns, nc = g.nc, e = g.e, e2 = 2 * g.e;
    const long total = (long)g.L * g.npairs * nc * nc * e2 * e2;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        long t = idx;
        const int qb = t % e2; t /= e2;
        const int qa = t % e2; t /= e2;
        const int d1 = t % nc; t /= nc;
        const int d2 = t % nc; t /= nc;
        const int pair = t % g.npairs;
        const int l = (int)(t / g.npairs);
        int i, ip;
        gram_pair(pair, Ns, i, ip);
        const int q2 = qa < e ? qa : n2 - e2 + qa, q1 = qb < e ? qb : n1 - e2 + qb;
        const double2* xi = x + ((size_t)l * Ns + i) * n2 * n1;
        const double2* xj = x + ((size_t)l * Ns + ip) * n2 * n1;
        cor[idx] = cconjmul(xi[(size_t)q2 * n1 + q1],
                            xj[(size_t)((q2 + d2 - e) & (n2 - 1)) * n1 + ((q1 + d1 - e) & (n1 - 1))]);
    }
}

// G[l][row][col] for row <= col (mirrored as the conjugate).  The band lines
// an anchor window at offset b misses are [0, b) and [e + b, 2e) in band order.
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
    const double2* ro = rows + o * e2;
    const double2* co = cols + o * e2;
    const double2* cr = cor + o * e2 * e2;
    double2 sr = cmk(0.0, 0.0), sc = cmk(0.0, 0.0), sx = cmk(0.0, 0.0);
    for (int q = 0; q < b2; ++q) sr = cadd(sr, ro[q]);
    for (int q = e + b2; q < e2; ++q) sr = cadd(sr, ro[q]);
    for (int q = 0; q < b1; ++q) sc = cadd(sc, co[q]);
    for (int q = e + b1; q < e2; ++q) sc = cadd(sc, co[q]);
    for (int seg = 0; seg < 2; ++seg) {
        const int qa0 = seg ? e + b2 : 0, qa1 = seg ? e2 : b2;
        for (int qa = qa0; qa < qa1; ++qa) {
            const double2* crow = cr + qa * e2;
            for (int qb = 0; qb < b1; ++qb) sx = cadd(sx, crow[qb]);
            for (int qb = e + b1; qb < e2; ++qb) sx = cadd(sx, crow[qb]);
        }
    }
    double2 v = cadd(csub(csub(C[o], sr), sc), sx);
    double2* Gl = G + (size_t)l * K * K;
    if (row == col) v.y = 0.0;
    Gl[(size_t)row * K + col] = v;
    if (row != col) Gl[(size_t)col * K + row] = cconj(v);
}
