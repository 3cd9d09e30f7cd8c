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

// Q as k_gram_q for n2 with an odd factor (3 or 7 times a power of two):
// the B columns at x inverse-transformed in shared memory (fft_batch_lds),
// then each (l, pair, d2) bin summed directly over n in order:
//   Q = (-1)^(d2-e) sum_n conj(u_i[n]) u_i'[n] w^{((d2-e) n) mod n2}.
// grid n1, block 512; shared memory (B + 1) n2 double2.
__global__ void __launch_bounds__(512)
k_gram_q_any(Geo g, const double2* __restrict__ h1, const double2* __restrict__ tw2, double2* __restrict__ Q) {
    extern __shared__ double2 sm[];
    const int n1 = g.n1, n2 = g.n2, B = g.B, Ns = g.Ns, nc = g.nc, e = g.e, npairs = g.npairs;
    const int x = blockIdx.x;
    double2* U = sm;                 // [B][n2]
    double2* TW = sm + B * n2;       // [n2]
    for (int k = threadIdx.x; k < n2; k += blockDim.x) TW[k] = tw2[k];
    for (int idx = threadIdx.x; idx < B * n2; idx += blockDim.x) {
        const int b = idx / n2, k = idx - b * n2;
        U[idx] = cscale(h1[((size_t)b * n1 + x) * n2 + k], sgn_pow(k));
    }
    fft_batch_lds(U, n2, g.logn2, B, n2, TW, true);
    const double isq = 1.0 / sqrt((double)n2);
    for (int idx = threadIdx.x; idx < B * n2; idx += blockDim.x) {
        const int n = idx % n2;
        U[idx] = cscale(U[idx], isq * sgn_pow(n));
    }
    __syncthreads();
    const int nt = g.L * npairs * nc;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
        const int task = t / nc, d2 = t - task * nc;
        const int l = task / npairs, pair = task - l * npairs;
        int i, ip;
        gram_pair(pair, Ns, i, ip);
        const double2* ui = U + (l * Ns + i) * n2;
        const double2* uj = U + (l * Ns + ip) * n2;
        const int step = imod(d2 - e, n2);
        double2 s = cmk(0.0, 0.0);
        int ph = 0;
        for (int n = 0; n < n2; ++n) {
            s = cfma(cconjmul(ui[n], uj[n]), TW[ph], s);
            ph += step;
            if (ph >= n2) ph -= n2;
        }
        Q[(((size_t)l * npairs + pair) * n1 + x) * nc + d2] = cscale(s, sgn_pow(d2 - e));
    }
}

// C[l][pair][d2][d1] = sum_x Q[l][pair][x][d2] e^{-2 pi i (d1-e)(x-n1/2)/n1}.
// One wave per (l, pair, d2): the wave's Q column and the kx twiddles are
// staged in shared memory in one batch, then lane = d1 + GS g sums the x of
// group g (fixed order) and the groups are added in order.
template <bool POW2>
__global__ void __launch_bounds__(256)
k_gram_c(Geo g, const double2* __restrict__ Q, const double2* __restrict__ tw1, double2* __restrict__ C) {
    __shared__ double2 qs[4][256];
    __shared__ double2 ts[256];
    const int n1 = g.n1, nc = g.nc, e = g.e;
    const int wl = threadIdx.x >> 6;
    const int wv = blockIdx.x * (blockDim.x >> 6) + wl;
    const int nwv = g.L * g.npairs * nc;
    const int lane = threadIdx.x & 63;
    const int lp = wv / nc, d2 = wv - lp * nc;      // lp = l * npairs + pair
    const bool live_wave = wv < nwv;
    const double2* q = Q + (size_t)(live_wave ? lp : 0) * n1 * nc + d2;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int x = lane + 64 * u;
        if (x < n1) qs[wl][x] = q[(size_t)x * nc];
        if (wl == 0 && x < n1) ts[x] = tw1[x];
    }
    __syncthreads();
    if (!live_wave) return;
    const int gs = gram_gs(nc), ng = 64 / gs;
    const int d1 = lane & (gs - 1), qg = lane / gs;
    const int xq = n1 / ng, x0 = qg * xq;
    double2 s = cmk(0.0, 0.0);
    if (d1 < nc) {
#pragma unroll 8
        for (int x = x0; x < x0 + xq; ++x) {
            const int ph = (d1 - e) * (x - n1 / 2);
            s = cfma(qs[wl][x], ts[POW2 ? ph & (n1 - 1) : imod(ph, n1)], s);
        }
    }
    s = gram_reduce_groups(s, gs);
    if (qg == 0 && d1 < nc) C[((size_t)lp * nc + d2) * nc + d1] = s;
}

// Band row and column sums of z_d.  One workgroup per (band line qa, l,
// pair) and kind (blockIdx.y: 0 rows, 1 columns):
//   rows[l][pair][d2][d1][qa] = sum_q1 conj(x_i[q2][q1]) x_i'[q2+d2-e][q1+d1-e],  q2 = band row qa
//   cols[l][pair][d2][d1][qa] = sum_q2 conj(x_i[q2][q1]) x_i'[q2+d2-e][q1+d1-e],  q1 = band col qa
// The line of x_i and the 2r-1 lines of x_i' it meets are staged in shared
// memory in one batch of loads (rows from the natural x, columns from the
// natural band columns xcol = pcol of x, contiguous in ky); each (fixed lag,
// free lag) is then summed by one thread from shared memory, in order.
// Dynamic shared memory: (1 + 2r-1) max(n1, n2) double2.
#define GRAM_STAGE 16
template <bool POW2>
__global__ void __launch_bounds__(256)
k_gram_lines(Geo g, const double2* __restrict__ x, const double2* __restrict__ xcol, double2* __restrict__ rows,
             double2* __restrict__ cols) {
    extern __shared__ double2 sm[];
    const int n1 = g.n1, n2 = g.n2, Ns = g.Ns, nc = g.nc, e = g.e, e2 = 2 * g.e;
    const bool col = blockIdx.y == 1;
    const int qa = blockIdx.x % e2, lp = blockIdx.x / e2, l = lp / g.npairs, pair = lp - l * g.npairs;
    int i, ip;
    gram_pair(pair, Ns, i, ip);
    const int n = col ? n2 : n1;
    double2* a = sm;           // [n]
    double2* b = sm + n;       // [nc][n]
    // stage: entry k < n is a[k]; entry n + f n + q is b[f][q].  Each entry is
    // base[line * ls + q] with the line picked arithmetically, so the loads of
    // a batch carry no branches and are all in flight together.
    const int q2a = qa < e ? qa : n2 - e2 + qa, q1a = qa < e ? qa : n1 - e2 + qa;
    const double2* base_i = col ? xcol + ((size_t)l * Ns + i) * 4 * e * n2 : x + ((size_t)l * Ns + i) * n2 * n1;
    const double2* base_j = col ? xcol + ((size_t)l * Ns + ip) * 4 * e * n2 : x + ((size_t)l * Ns + ip) * n2 * n1;
    const int ls = col ? n2 : n1;
    const int line_a = col ? band_pcol(q1a, n1, e) : q2a;
    const int tot = (1 + nc) * n;
    for (int base = threadIdx.x; base < tot; base += GRAM_STAGE * blockDim.x) {
        double2 v[GRAM_STAGE];
#pragma unroll
        for (int u = 0; u < GRAM_STAGE; ++u) {
            const int k0 = base + u * blockDim.x, k = k0 < tot ? k0 : tot - 1;
            const bool isa = k < n;
            const int f = isa ? 0 : (k - n) / n, q = isa ? k : (k - n) - f * n;
            const int line_b = col ? band_pcol(POW2 ? (q1a + f - e) & (n1 - 1) : wrap1(q1a + f - e, n1), n1, e)
                                   : (POW2 ? (q2a + f - e) & (n2 - 1) : wrap1(q2a + f - e, n2));
            const double2* bp = isa ? base_i : base_j;
            v[u] = bp[(size_t)(isa ? line_a : line_b) * ls + q];
        }
#pragma unroll
        for (int u = 0; u < GRAM_STAGE; ++u) {
            const int k0 = base + u * blockDim.x;
            sm[k0 < tot ? k0 : tot - 1] = v[u];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nc * nc; t += blockDim.x) {
        const int fx = t / nc, fr = t - fx * nc;   // fixed lag, free lag
        const double2* bf = b + (size_t)fx * n;
        // four interleaved partial sums (q mod 4), added in a fixed order at the end
        double2 s4[4] = {cmk(0.0, 0.0), cmk(0.0, 0.0), cmk(0.0, 0.0), cmk(0.0, 0.0)};
        // a is the same for every thread: read it from global memory through the
        // constant address space (scalar loads) instead of shared memory
        const __attribute__((address_space(4))) double* a4 =
            (const __attribute__((address_space(4))) double*)(uintptr_t)(base_i + (size_t)line_a * ls);
#pragma unroll 2
        for (int q = 0; q < n; q += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = q + u + fr - e;
                s4[u] = cfma(cmk(a4[2 * (q + u)], -a4[2 * (q + u) + 1]), bf[POW2 ? j & (n - 1) : wrap1(j, n)], s4[u]);
            }
        }
        const double2 s = cadd(cadd(s4[0], s4[1]), cadd(s4[2], s4[3]));
        const int d2 = col ? fr : fx, d1 = col ? fx : fr;
        (col ? cols : rows)[(((size_t)lp * nc + d2) * nc + d1) * e2 + qa] = s;
    }
}

// Corner values cor[l][pair][d2][d1][qa][qb] = z_d[band row qa][band col qb].
template <bool POW2>
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
                            xj[(size_t)(POW2 ? (q2 + d2 - e) & (n2 - 1) : wrap1(q2 + d2 - e, n2)) * n1 +
                               (POW2 ? (q1 + d1 - e) & (n1 - 1) : wrap1(q1 + d1 - e, n1))]);
    }
}

// G[l][row][col] for row <= col (mirrored as the conjugate).  The band lines
// an anchor window at offset b misses are [0, b) and [e + b, 2e) in band order.
// One 64-thread workgroup per lag group o = (l, pair, d2, d1): its band row,
// column and corner sums are staged in shared memory once, then each thread
// assembles the entries (b2, b1) of the group, summing in band order.
__global__ void __launch_bounds__(64)
k_gram_assemble(Geo g, const double2* __restrict__ C, const double2* __restrict__ rows,
                const double2* __restrict__ cols, const double2* __restrict__ cor, double2* __restrict__ G) {
    __shared__ double2 rs[16], cs[16], xs[256];
    const int K = g.K, r = g.r, Ns = g.Ns, nc = g.nc, e = g.e, e2 = 2 * g.e;
    const int o = blockIdx.x;                         // ((l npairs + pair) nc + d2) nc + d1
    const int d1 = o % nc, d2 = (o / nc) % nc, lp = o / (nc * nc);
    const int l = lp / g.npairs, pair = lp - l * g.npairs;
    int i, ip;
    gram_pair(pair, Ns, i, ip);
    if (threadIdx.x < e2) {
        rs[threadIdx.x] = rows[(size_t)o * e2 + threadIdx.x];
        cs[threadIdx.x] = cols[(size_t)o * e2 + threadIdx.x];
    }
    for (int k = threadIdx.x; k < e2 * e2; k += blockDim.x) xs[k] = cor[(size_t)o * e2 * e2 + k];
    const double2 c0 = C[o];
    __syncthreads();
    double2* Gl = G + (size_t)l * K * K;
    for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
        const int b2 = t / r, b1 = t - b2 * r;
        const int c2 = b2 + d2 - e, c1 = b1 + d1 - e;
        if (c2 < 0 || c2 >= r || c1 < 0 || c1 >= r) continue;
        const int row = (i * r + b2) * r + b1, col = (ip * r + c2) * r + c1;
        if (row > col) continue;
        double2 sr = cmk(0.0, 0.0), sc = cmk(0.0, 0.0), sx = cmk(0.0, 0.0);
        for (int q = 0; q < b2; ++q) sr = cadd(sr, rs[q]);
        for (int q = e + b2; q < e2; ++q) sr = cadd(sr, rs[q]);
        for (int q = 0; q < b1; ++q) sc = cadd(sc, cs[q]);
        for (int q = e + b1; q < e2; ++q) sc = cadd(sc, cs[q]);
        for (int seg = 0; seg < 2; ++seg) {
            const int qa0 = seg ? e + b2 : 0, qa1 = seg ? e2 : b2;
            for (int qa = qa0; qa < qa1; ++qa) {
                const double2* crow = xs + qa * e2;
                for (int qb = 0; qb < b1; ++qb) sx = cadd(sx, crow[qb]);
                for (int qb = e + b1; qb < e2; ++qb) sx = cadd(sx, crow[qb]);
            }
        }
        double2 v = cadd(csub(csub(c0, sr), sc), sx);
        if (row == col) v.y = 0.0;
        Gl[(size_t)row * K + col] = v;
        if (row != col) Gl[(size_t)col * K + row] = cconj(v);
    }
}
