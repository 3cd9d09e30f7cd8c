// Conjugate gradients on the hybrid layout (x image, ky k-space): the normal
// operator's column pass works there, and the kx transform is unitary, so the
// CG iterates are the transformed natural-domain iterates (inner products and
// step lengths unchanged).  The only natural-domain work left is on the band
// (pixels within e of an edge): its columns are taken from the hybrid vector
// here, and its corrections are injected back in the CG update.
#pragma once
#include "smsm_dense.h"

#define EXTRACT_WAVES 8                      // waves per workgroup of k_band_extract (split x)
#define EXTRACT_KS (64 / EXTRACT_WAVES)      // k steps (4 x each) per wave at most (n1 <= 256)

// Natural columns of p within 2e of the kx edges:
//   pcol[b][c][ky] = sum_x fx[x][c] pt[b][x][ky],
//   fx[x][c] = e^{-2 pi i (kx_c - n1/2)(x - n1/2)/n1} / sqrt(n1),
//   kx_c = c for c < 2e, n1 - 4e + c otherwise (fx is zero for c >= 4e).
// One 16 (ky) x 16 (c) tile per workgroup on FP64 matrix cores: lane l
// supplies pt[b][x0 + l/16][ky0 + l%16] (16 contiguous ky) and
// fx[x0 + l/16][c0 + l%16]; 4 waves split x; partial tiles summed in order.
// With write_prow, the workgroups of the first c tile also copy the hybrid
// rows within 2e of the ky edges, transposed: prow[b][j][x], j = ky for
// ky < 2e, else ky - (n2 - 4e) (the band rows' kx taps then read contiguous
// x); the fast column pass writes that copy itself.
// grid (n2/16 * np/16, B), block 64 EXTRACT_WAVES; np = padded width of fx.
// The c tile varies slowest within a row of the grid, so the workgroups that
// read the same 16 ky of p are n2/16 ids apart (a multiple of 8 for n2 >= 128:
// the same XCD, whose L2 then serves the second read).
__global__ void __launch_bounds__(64 * EXTRACT_WAVES)
k_band_extract(int n1, int n2, int e, int np, const double2* __restrict__ pt, const double2* __restrict__ fx,
               double2* __restrict__ pcol, double2* __restrict__ prow, int write_prow) {
    __shared__ double acc[EXTRACT_WAVES][8][64];
    const int b = blockIdx.y;
    const int nmt = n2 / 16, t = blockIdx.x, ct = t / nmt, mt = t - ct * nmt;
    const int ky0 = mt * 16, c0 = ct * 16;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), kq = lane >> 4;
    const double2* Ap = pt + ((size_t)b * n1 + kq) * n2 + ky0 + (lane & 15);   // pt[b][x][ky]
    const double2* Bp = fx + (size_t)kq * np + c0 + (lane & 15);               // fx[x][c]
    // k steps of 4 x per wave: nks / 4 <= EXTRACT_KS (n1 <= 256); every load
    // of the wave is issued before the first product
    const int nks = n1 / 4, ks0 = (w * nks) / EXTRACT_WAVES, ks1 = ((w + 1) * nks) / EXTRACT_WAVES;
    // complex product with three real products (Gauss):
    //   t1 = (ar + ai) br, t2 = ar (bi - br), t3 = ai (br + bi); re = t1 - t3, im = t1 + t2
    hd4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = {0.0, 0.0, 0.0, 0.0}, t3 = {0.0, 0.0, 0.0, 0.0};
    double2 av[EXTRACT_KS], bv[EXTRACT_KS];
#pragma unroll
    for (int u = 0; u < EXTRACT_KS; ++u) {
        const int k = 4 * max(min(ks0 + u, ks1 - 1), 0);   // a wave with no k step reads row 0
        av[u] = Ap[(size_t)k * n2];
        bv[u] = Bp[(size_t)k * np];
    }
    if (write_prow && ct == 0) {
        const int ky = ky0 + (lane & 15);
        if (ky < 2 * e || ky >= n2 - 2 * e) {
            const int j = ky < 2 * e ? ky : ky - (n2 - 4 * e);
#pragma unroll
            for (int u = 0; u < EXTRACT_KS; ++u)
                if (ks0 + u < ks1) prow[((size_t)b * 4 * e + j) * n1 + 4 * (ks0 + u) + kq] = av[u];
        }
    }
#pragma unroll
    for (int u = 0; u < EXTRACT_KS; ++u) {
        if (ks0 + u < ks1) {
            t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x + av[u].y, bv[u].x, t1, 0, 0, 0);
            t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv[u].y - bv[u].x, t2, 0, 0, 0);
            t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].y, bv[u].x + bv[u].y, t3, 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        acc[w][v][lane] = t1[v] - t3[v];
        acc[w][4 + v][lane] = t1[v] + t2[v];
    }
    __syncthreads();
    if (threadIdx.x < 256) {   // one thread per tile element: register v of lane ln
        const int v = threadIdx.x >> 6, ln = threadIdx.x & 63;
        double2 c = cmk(0.0, 0.0);
#pragma unroll
        for (int ww = 0; ww < EXTRACT_WAVES; ++ww) {
            c.x += acc[ww][v][ln];
            c.y += acc[ww][4 + v][ln];
        }
        const int ky = ky0 + 4 * v + (ln >> 4), col = c0 + (ln & 15);
        if (col < 4 * e) pcol[((size_t)b * 4 * e + col) * n2 + ky] = c;
    }
}

// Vector pass on the hybrid layout after the column pass (and the band
// kernel when BAND): q = h2 + band correction, then
//   mode 0: out = q
//   mode 1: out = bvec - q (CG residual); per-block partials of |out|^2
//   mode 2: CG step r -= alpha q; partials of |r|^2 (x takes alpha p in the
//           next column pass, or in k_x_step after the last step).  Wave 0
//           of every workgroup forms alpha = *rr / sum(pq[0..npq)) before
//           its own vector loads and shares it through shared memory (the
//           same fixed-order sum everywhere, so all workgroups agree);
//           rr == 0 (exact solution) gives alpha = 0, a non-finite |r|^2
//           or a non-positive or non-finite curvature gives alpha = 0 and
//           sets flags[0]; the
//           first workgroup stores alpha in *alpha_out.
// Thread layout: lane = ky (LY = min(64, n2) lanes per x, 64 / LY x per
// step), so the natural band-column corrections of a lane's ky (shares
// summed, corner cross terms added; staged once per workgroup) stay in
// registers while the wave takes XW steps of x; with one x per step (WU) the
// kx inverse-transform coefficients finv[x][.] are wave-uniform.  All global
// loads of a thread are unconditional and issued before the first use.
// grid (n2 / LY * n1 / (4 XW (64 / LY)), B), block 256; one partial per block.
struct HybArgs {
    Geo g;
    int mode, use_band;
    const double2* h2;
    const double2* bvec;
    double2* out;
    double2* r;
    BandInj bi;
    const double* rr;        // |r|^2 of the current residual (mode 2, scalar)
    const double* pq;        // partials of Re <p, N p> (mode 2): column pass, then band
    int npq;
    double* alpha_out;       // the step length (mode 2, written by the first workgroup)
    int* flags;
    double* part;            // per-block partials of |r|^2
};

#define HYB_MAX_E2 16
#define HYB_CONST __attribute__((address_space(4)))
#define HYB_WAVES 4   // waves per workgroup of the vector pass
#define HYB_CS_PER_THREAD (HYB_MAX_E2 / HYB_WAVES)   // staged corrections per thread (HYB_MAX_E2 x 64 entries)
template <int MODE, int XW, bool WU, bool BAND>
__global__ void __launch_bounds__(64 * HYB_WAVES) k_hyb_update(HybArgs a) {
    __shared__ double red[8];
    __shared__ double alpha_sh;
    __shared__ double2 cs[BAND ? HYB_MAX_E2 * 64 : 1];    // corrections [cl][ky in chunk]
    const Geo& g = a.g;
    const int n1 = g.n1, n2 = g.n2, e = g.e, e2 = 2 * g.e;
    const int LY = min(64, n2 & -n2), XPS = 64 / LY, nkc = n2 / LY;   // ky chunk: largest power of two dividing n2, <= 64
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int kc = blockIdx.x % nkc, xb = blockIdx.x / nkc, b = blockIdx.y;
    const int ky = kc * LY + lane % LY, xs = lane / LY;
    const int x0 = (xb * HYB_WAVES + wave) * XW * XPS;
    const double2* __restrict__ h2 = a.h2;
    double2* __restrict__ rv = a.r;
    double2* __restrict__ out = a.out;
    const bool rb = ky < e || ky >= n2 - e;            // this lane's ky is a band row
    const int rrow = rb ? (ky < e ? ky : ky - (n2 - e2)) : 0;

    // ---- step length (wave 0, before its vector loads)
    if (MODE == 2 && wave == 0) {
        const double pq = wave_sum_partials(a.pq, a.npq, lane), rr = *a.rr;
        const double al = rr / pq;
        // a non-finite |r|^2 (NaN or Inf reached the residual) is flagged, not
        // taken for an exact solution
        const bool bad = !isfinite(rr) || (rr > 0.0 && (!(pq > 0.0) || !isfinite(al)));
        const double alpha0 = (rr > 0.0 && !bad) ? al : 0.0;
        if (lane == 0) {
            alpha_sh = alpha0;
            if (blockIdx.x == 0 && blockIdx.y == 0) {
                *a.alpha_out = alpha0;
                if (bad) a.flags[0] = 1;
            }
        }
    }

    // ---- band-column corrections of this workgroup's ky: shares and corner terms
    double2 cv[HYB_CS_PER_THREAD];
    if (BAND) {
        const int ncs = e2 * LY, ds = a.bi.ds;
#pragma unroll
        for (int u = 0; u < HYB_CS_PER_THREAD; ++u) {
            const int idx0 = threadIdx.x + u * 64 * HYB_WAVES;
            const int idx = idx0 < ncs ? idx0 : ncs - 1;
            const int cl = idx / LY, kyl = idx - cl * LY, kyc = kc * LY + kyl;
            double2 v[BAND_MAX_DS];
#pragma unroll
            for (int part = 0; part < BAND_MAX_DS; ++part)
                v[part] = a.bi.ccol[(((size_t)(part < ds ? part : ds - 1) * g.B + b) * e2 + cl) * n2 + kyc];
            const bool crn = kyc < e || kyc >= n2 - e;
            const int corner = (kyc < e ? 0 : 1) | (cl < e ? 0 : 2);
            const int rrc = crn ? (kyc < e ? kyc : kyc - (n2 - e)) : 0, cc = cl < e ? cl : cl - e;
            const double2 cn = a.bi.ccorner[(size_t)b * 4 * e * e + corner * e * e + rrc * e + cc];
            double2 sum = cscale(cn, crn ? 1.0 : 0.0);
#pragma unroll
            for (int part = 0; part < BAND_MAX_DS; ++part) sum = cadd(sum, cscale(v[part], part < ds ? 1.0 : 0.0));
            cv[u] = sum;
        }
    }
    // ---- vectors
    int xx[XW];
    size_t kk[XW];
    double2 q[XW], v1[XW], v3[XW], cr[XW];
#pragma unroll
    for (int t = 0; t < XW; ++t) {
        xx[t] = x0 + t * XPS + xs;
        if (WU) xx[t] = __builtin_amdgcn_readfirstlane(xx[t]);
        kk[t] = ((size_t)b * n1 + xx[t]) * n2 + ky;
        q[t] = h2[kk[t]];
        if (MODE == 1) v1[t] = a.bvec[kk[t]];
        if (MODE == 2) v3[t] = rv[kk[t]];
        if (BAND) cr[t] = a.bi.crow[((size_t)b * e2 + rrow) * n1 + xx[t]];
    }
    if (MODE == 2 && !BAND) __syncthreads();          // alpha_sh (BAND: the staging barrier below)
    double2 c[HYB_MAX_E2];
    if (BAND) {
        const int ncs = e2 * LY;
        // (threads past the end rewrite the last entry with its own value)
#pragma unroll
        for (int u = 0; u < HYB_CS_PER_THREAD; ++u) {
            const int i0 = threadIdx.x + u * 64 * HYB_WAVES;
            const int ic = i0 < ncs ? i0 : ncs - 1, cl = ic / LY, kyl = ic - cl * LY;
            cs[cl * 64 + kyl] = cv[u];
        }
        __syncthreads();
#pragma unroll
        for (int cl = 0; cl < HYB_MAX_E2; ++cl) c[cl] = cl < e2 ? cs[cl * 64 + lane % LY] : cmk(0.0, 0.0);
    }
    const double alpha = MODE == 2 ? alpha_sh : 0.0;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < XW; ++t) {
        double2 qt = q[t];
        if (BAND) {
            // finv rows are HYB_MAX_E2 wide, zero past 2e
            if (WU) {
                // finv is constant while the kernel runs: wave-uniform reads
                // through the constant address space (scalar loads)
                const HYB_CONST double* fx =
                    (const HYB_CONST double*)(uintptr_t)(a.bi.finv + (size_t)xx[t] * HYB_MAX_E2);
#pragma unroll
                for (int cl = 0; cl < HYB_MAX_E2; ++cl) qt = cfma(cmk(fx[2 * cl], fx[2 * cl + 1]), c[cl], qt);
            } else {
                const double2* fx = a.bi.finv + (size_t)xx[t] * HYB_MAX_E2;
#pragma unroll
                for (int cl = 0; cl < HYB_MAX_E2; ++cl) qt = cfma(fx[cl], c[cl], qt);
            }
            qt = cadd(qt, cscale(cr[t], rb ? 1.0 : 0.0));
        }
        if (MODE == 0) {
            out[kk[t]] = qt;
        } else if (MODE == 1) {
            const double2 v = csub(v1[t], qt);
            out[kk[t]] = v;
            s += cabs2(v);
        } else {
            const double2 v = csub(v3[t], cscale(qt, alpha));
            rv[kk[t]] = v;
            s += cabs2(v);
        }
    }
    if (MODE != 0) {
        s = block_sum(s, red);
        if (threadIdx.x == 0) a.part[blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

// p = r (first step) or p = r + beta p_old, beta = sum rr_new[0..nrr) /
// *rr_old, for column passes that do not fuse the update (p_old may be p),
// with the previous step x += (*alpha_prev) p_old when x is given; the first
// block stores sum rr_new[0..nrr) (the new |r|^2) in *rr_out.
__global__ void k_hyb_pupdate(long n, const double2* __restrict__ r, const double2* p_old, double2* p,
                              double2* __restrict__ x, const double* __restrict__ alpha_prev,
                              const double* __restrict__ rr_new, int nrr, const double* __restrict__ rr_old,
                              double* __restrict__ rr_out, int first) {
    __shared__ double red[8];
    double beta = 0.0;
    const double ap = (!first && x) ? *alpha_prev : 0.0;
    const double rn = sum_partials(rr_new, nrr, red);
    if (!first) {
        const double ro = *rr_old;
        beta = ro > 0.0 ? rn / ro : 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *rr_out = rn;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        if (first) {
            p[k] = r[k];
        } else {
            const double2 po = p_old[k];
            if (x) x[k] = cadd(x[k], cscale(po, ap));
            p[k] = cadd(r[k], cscale(po, beta));
        }
}

// x += (*alpha) p: the last CG step of a cycle (the earlier steps reach x
// in the column pass that follows them).
__global__ void k_x_step(long n, double2* __restrict__ x, const double2* __restrict__ p,
                         const double* __restrict__ alpha) {
    const double al = *alpha;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        x[k] = cadd(x[k], cscale(p[k], al));
}

// Per-block partials of Re <p, q>.
__global__ void k_hyb_dot(long n, const double2* __restrict__ p, const double2* __restrict__ q,
                          double* __restrict__ part) {
    __shared__ double red[16];
    double s = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const double2 a = p[k], b = q[k];
        s += a.x * b.x + a.y * b.y;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}
