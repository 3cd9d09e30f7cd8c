// Host side of the SMS-MUSSELS solver: plan creation, device memory layout,
// and the kernel sequences behind every C-ABI entry point of smsm.h.
#include "smsm_kernels.h"
#include "smsm_col_fast.h"
#include "smsm_col_mix.h"
#include "smsm_wavefft.h"
#include "smsm_dense.h"
#include "smsm_gram.h"
#include "smsm_hyb.h"
#include "smsm_cnn.h"
#include "smsm_cnn_mfma.h"
#include "smsm_al.h"
#include "smsm_gram_mfma.h"
#include "smsm.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

namespace {

constexpr int kThreads = 256;
constexpr int kColThreads = 512;
constexpr int kVecBlocks = 512;      // fixed grid of the CG vector kernels
constexpr int kNsDefaultIters = 16;  // Newton-Schulz iteration cap
constexpr int kSqSteps = 30;         // squarings for the largest eigenvalue
constexpr int kPadBlocks = 32;       // blocks per slice of the dense set-up kernels
constexpr double kNsTol = 1e-10;     // ||I - Z Y||_F at which NS is converged
constexpr int kBatchMaxRepeat = 5;   // entries of one plan per captured graph of a batch
constexpr int kBatchMaxSegment = 30; // entries per captured graph of a batch

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
// log2 of the largest power of two dividing v (v > 0): the radix-2 part of a
// transform length
int pow2_log(int v) {
    int l = 0;
    while (((v >> l) & 1) == 0) ++l;
    return l;
}
// transform lengths the kernels take: 16 .. 256, a power of two times 1, 3 or
// 7, and a multiple of 16
bool length_ok(int n) {
    if (n < 16 || n > 256 || n % 16 != 0) return false;
    const int q = n >> pow2_log(n);
    return q == 1 || q == 3 || q == 7;
}
constexpr int kRowsAnyTR = 8;         // rows per workgroup of the row passes for lengths with an odd factor
// ky chunk of the hybrid vector pass: the largest power of two dividing n2, at most 64
int hyb_ly(const Geo& g) { return std::min(64, g.n2 & -g.n2); }
// Patch-anchor geometry of the Hankel matrices (the GEMM-form Gram and the
// augmented-Lagrangian kernels)
AlGeo anchor_geo(const Geo& g) {
    AlGeo a{};
    a.n1 = g.n1; a.n2 = g.n2; a.L = g.L; a.Ns = g.Ns; a.r = g.r; a.K = g.K; a.KP = dense_stride(g.K);
    a.P1 = g.n1 - g.r + 1; a.P2 = g.n2 - g.r + 1; a.NP = a.P1 * a.P2;
    a.NPP = (a.NP + AL_PT - 1) / AL_PT * AL_PT;
    a.KB = (g.K + AL_BK - 1) / AL_BK;
    return a;
}
int gram_bf16_chunks(const AlGeo& a) { return (a.NP + GB_CH - 1) / GB_CH; }

// Offsets (bytes from the workspace base) of the buffers a solve writes.
struct WsLayout {
    size_t x, b, r, p, q, h1, h2, ytil, G, W, Y0, Y1, Z0, Z1, T, Kc, Khat, Dside, Dx, crow, ccol, ccorner, Dhat,
        pcol, prow, gpart, gC, grow, gcol, gcor, pr, pq, part0, part1, sigma, eps, wscale, epsin, nsmu, done, cgs,
        gbpart;
};

}  // namespace

struct smsm_plan {
    Geo g;
    smsm_params prm;
    int dev = 0;
    int TR = 1, TRy = 1;
    int TRw = 8;              // rows per workgroup of the in-wave FFT row passes
    int rows_blk = 256;       // threads per workgroup of the row passes
    size_t lds_roww = 0;
    int npc = 0;             // partials of Re <p, column pass> (one per column workgroup, or kVecBlocks)
    int npr = 0;             // partials of |r|^2 (blocks of the hybrid vector pass)
    int npr_max = 0;         // the largest npr of any vector-pass shape (size of the ring)
    int hyb_xw = 1;          // x steps per wave of the hybrid vector pass
    dim3 hyb_grid;
    int np_band = 0;         // padded width of the band-column extraction table
    int KP = 0;              // padded stride of the Newton-Schulz matrices
    int ntile = 0;           // 16x16 tiles per slice of the dense products
    int npmax = 0;           // partial sums per slice (max over producers)
    size_t lds_rows = 0, lds_col = 0, lds_gram = 0, lds_gram_lines = 0;
    bool have_weights = false;
    bool khat_f32 = false;   // Khat, Dhat and Dx were last built as complex64 (SMSM_FLAG_REG_F32)
    void* arena = nullptr;   // plan-owned: what creation derives (coil maps, tables, status word)
    size_t bytes = 0;
    void* ws = nullptr;      // caller-owned workspace (every buffer a solve writes), or null
    size_t ws_bytes = 0;     // bytes the workspace must hold
    WsLayout wo{};           // offsets of the scratch buffers in the workspace
    // device buffers (plan arena)
    double2* ST = nullptr;                    // coils [L][Nc][n1][n2], complex128
    double2 *tw1 = nullptr, *tw2 = nullptr, *twM = nullptr;
    double2 *theta = nullptr, *tau = nullptr;
    int* flags = nullptr;    // numeric status: [0] CG curvature non-finite or <= 0, [1] weights not converged
    // device buffers (workspace)
    double2 *x = nullptr, *b = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
    double2 *h1 = nullptr, *h2 = nullptr, *ytil = nullptr;
    double2 *G = nullptr, *W = nullptr, *Y0 = nullptr, *Y1 = nullptr, *Z0 = nullptr, *Z1 = nullptr, *T = nullptr;
    double2* gbpart = nullptr;   // chunk partials of the GEMM-form Gram
    bool gram_bf16_ws = false;   // the workspace holds gbpart (created with SMSM_FLAG_GRAM_BF16)
    double2 *Kc = nullptr, *Khat = nullptr, *Dside = nullptr, *Dx = nullptr, *crow = nullptr, *ccol = nullptr, *ccorner = nullptr;
    double2 *Dhat = nullptr, *pcol = nullptr, *prow = nullptr, *fx = nullptr, *finv = nullptr;
    double2 *gpart = nullptr, *gC = nullptr, *grow = nullptr, *gcol = nullptr, *gcor = nullptr;
    double *pr = nullptr, *pq = nullptr, *bpart = nullptr, *part0 = nullptr, *part1 = nullptr, *sigma = nullptr, *eps = nullptr;
    double *wscale = nullptr, *epsin = nullptr, *nsmu = nullptr;
    double* cgs = nullptr;   // CG scalars: |r|^2 of the last three residuals [0..2]; the last step length [8]
    int* done = nullptr;

    int ns_iters = kNsDefaultIters;
    int col_fast = -1;        // instance of k_col_fast for this geometry (-1: generic k_col)
    int col_mix = -1;         // instance of k_col_mix (odd-factor folded lengths) for the normal pass, or -1
    size_t lds_colmix = 0;
    // per-launch timing of the fast column pass (diagnostic, off by default):
    // start/stop event pairs recorded with the dispatches
    std::vector<hipEvent_t> kt_ev;
    int kt_cap = 0, kt_n = 0, kt_stride = 1, kt_seen = 0;
    size_t lds_colfast = 0;
    size_t lds_band = 0;
    BandFn band = nullptr;   // band-correction kernel for (2r-1, Ns)
    BandFn band_f32 = nullptr;   // the same reading complex64 tables (SMSM_FLAG_REG_F32)
};

namespace {

#define LAUNCH_CHECK()                                      \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return SMSM_E_DEVICE; \
    } while (0)

smsm_status check_params(const smsm_params* p) {
    if (!p) return SMSM_E_INVALID;
    if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return SMSM_E_INVALID;
    if (p->n_irls < 1 || p->n_cg < 0) return SMSM_E_INVALID;
    if (!(p->eps_frac > 0.0) || !(p->eps_decay >= 1.0) || !(p->eps_floor_frac >= 0.0)) return SMSM_E_INVALID;
    if (p->ns_max_iter < 0 || p->ns_max_iter > 200) return SMSM_E_INVALID;
    return SMSM_OK;
}

void twiddles(int n, std::vector<double2>& out) {
    out.resize(n);
    for (int k = 0; k < n; ++k) {
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)n;
        out[k] = make_double2((double)cosl(a), (double)sinl(a));
    }
}

// Carve 256-byte aligned pieces out of one allocation.
struct Carver {
    size_t off = 0;
    template <class T>
    size_t take(size_t count) {
        const size_t o = (off + 255) & ~size_t(255);
        off = o + count * sizeof(T);
        return o;
    }
};

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

dim3 vec_grid() { return dim3(kVecBlocks); }

// Launch shapes a plan can take (smsm_plan_autotune picks among them).
// Row transforms: TRw rows per workgroup; the kernel needs TRw a multiple of
// (waves per workgroup) x (rows per wave) and TRw n1 <= 8 x threads.
bool rows_shape_ok(const Geo& g, int trw) {
    const int G = std::max(1, 64 / g.n1), blk = std::min(256, 64 * trw / G);
    return trw >= 1 && g.n2 % trw == 0 && blk >= 64 && trw % ((blk / 64) * G) == 0 && trw * g.n1 <= 8 * blk;
}
void set_rows_shape(smsm_plan* P, int trw) {
    const int n1 = P->g.n1;
    P->TRw = trw;
    P->rows_blk = std::min(256, 64 * trw / std::max(1, 64 / n1));
    P->lds_roww = (size_t)trw * (n1 + 1) * sizeof(double2) + 16 * sizeof(double);
}
// Vector pass: xw columns per wave, HYB_WAVES waves per workgroup, chunks of
// min(n2, 64) ky; the blocks must tile the image exactly.
int hyb_blocks(const Geo& g, int xw) {
    const int LY = hyb_ly(g), XPS = 64 / LY, per = HYB_WAVES * xw * XPS;
    if (g.n1 % per != 0) return 0;
    return (g.n2 / LY) * (g.n1 / per) * g.B;
}
bool set_hyb_shape(smsm_plan* P, int xw) {
    const Geo& g = P->g;
    const int nb = hyb_blocks(g, xw);
    if (nb <= 0 || (P->npr_max > 0 && nb > P->npr_max)) return false;
    const int LY = hyb_ly(g), XPS = 64 / LY;
    P->hyb_xw = xw;
    P->hyb_grid = dim3((g.n2 / LY) * (g.n1 / (HYB_WAVES * xw * XPS)), g.B);
    P->npr = nb;
    return true;
}

// ---- kernel chains -------------------------------------------------------
// kx inverse DFT, natural [B][n2][n1] -> hybrid [B][n1][n2].
smsm_status rows_inv(smsm_plan* P, const double2* in, double2* out, hipStream_t st) {
    const Geo& g = P->g;
    if (!is_pow2(g.n1)) {
        hipLaunchKernelGGL(k_rows_any<true>, dim3(g.n2 / kRowsAnyTR, g.B), dim3(kThreads),
                           (size_t)kRowsAnyTR * (g.n1 + 1) * sizeof(double2), st, g, in, out, P->tw1, kRowsAnyTR);
        LAUNCH_CHECK();
        return SMSM_OK;
    }
    const dim3 grid(g.n2 / P->TRw, g.B), blk(P->rows_blk);
    const size_t lds = P->lds_roww;
    switch (g.n1) {
        case 16: hipLaunchKernelGGL(k_rows_inv_w<16>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
        case 32: hipLaunchKernelGGL(k_rows_inv_w<32>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
        case 64: hipLaunchKernelGGL(k_rows_inv_w<64>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
        case 128: hipLaunchKernelGGL(k_rows_inv_w<128>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
        default: hipLaunchKernelGGL(k_rows_inv_w<256>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
    }
    LAUNCH_CHECK();
    return SMSM_OK;
}

// kx forward DFT, hybrid -> natural.
smsm_status rows_fwd(smsm_plan* P, const double2* in, double2* out, hipStream_t st) {
    const Geo& g = P->g;
    if (!is_pow2(g.n1)) {
        hipLaunchKernelGGL(k_rows_any<false>, dim3(g.n2 / kRowsAnyTR, g.B), dim3(kThreads),
                           (size_t)kRowsAnyTR * (g.n1 + 1) * sizeof(double2), st, g, in, out, P->tw1, kRowsAnyTR);
        LAUNCH_CHECK();
        return SMSM_OK;
    }
    const dim3 grid(g.n2 / P->TRw, g.B), blk(P->rows_blk);
    const size_t lds = P->lds_roww;
    switch (g.n1) {
        case 16: hipLaunchKernelGGL(k_rows_fwd_w<16>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
        case 32: hipLaunchKernelGGL(k_rows_fwd_w<32>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
        case 64: hipLaunchKernelGGL(k_rows_fwd_w<64>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
        case 128: hipLaunchKernelGGL(k_rows_fwd_w<128>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
        default: hipLaunchKernelGGL(k_rows_fwd_w<256>, grid, blk, lds, st, g, in, out, P->tw1, P->TRw); break;
    }
    LAUNCH_CHECK();
    return SMSM_OK;
}

// Instances of the register-resident column kernel: (M, L, Ns) with two
// coil-group waves per shot.
struct ColFastInst {
    int M, L, Ns;
    const void* fn;
    const void* fn_f32;   // the instance reading Khat as complex64
};
// Instances: 4 shots with two coil groups (8 waves), 8 shots with one (8
// waves, two or four coils per wave), 2 shots with four (8 waves; at folded
// length 128 two points per lane); the folded length M = n2 / Ns.
#define COLFAST(M_, L_, NS_, CG_) \
    {M_, L_, NS_, (const void*)&k_col_fast<M_, L_, NS_, CG_>, (const void*)&k_col_fast<M_, L_, NS_, CG_, true>}
const ColFastInst kColFast[] = {COLFAST(16, 2, 4, 2),  COLFAST(16, 3, 4, 2),  COLFAST(32, 2, 4, 2),
                                COLFAST(32, 3, 4, 2),  COLFAST(64, 2, 4, 2),  COLFAST(64, 3, 4, 2),
                                COLFAST(32, 2, 8, 1),  COLFAST(16, 2, 8, 1),  // (three slices at 8 shots spill)
                                COLFAST(128, 2, 2, 4), COLFAST(128, 3, 2, 4), COLFAST(64, 2, 2, 4),
                                COLFAST(64, 3, 2, 4)};
#undef COLFAST

// Normal-pass instances for folded lengths with an odd factor (8 waves).
struct ColMixInst {
    int M, L, Ns, CG;
    const void* fn;
};
#define COLMIX(M_, L_, NS_, CG_) {M_, L_, NS_, CG_, (const void*)&k_col_mix<M_, L_, NS_, CG_>}
const ColMixInst kColMix[] = {COLMIX(56, 3, 4, 2),  COLMIX(56, 2, 4, 2),  COLMIX(48, 3, 4, 2),  COLMIX(48, 2, 4, 2),
                              COLMIX(28, 2, 8, 1),  COLMIX(24, 2, 8, 1),  COLMIX(28, 2, 4, 2),  COLMIX(112, 2, 2, 4),
                              COLMIX(96, 3, 2, 4),  COLMIX(96, 2, 2, 4),  COLMIX(112, 3, 2, 4)};
#undef COLMIX

template <int M_, int L_, int NS_, int CG_, bool KF32>
void launch_colfast_k(smsm_plan* P, const double2* in, double2* out, int use_reg, const ColCg& pc, hipStream_t st) {
    const Geo& g = P->g;
    if (P->kt_n < P->kt_cap && P->kt_seen++ % P->kt_stride == 0) {
        const int n = P->kt_n++;
        hipExtLaunchKernelGGL((k_col_fast<M_, L_, NS_, CG_, KF32>), dim3(g.n1), dim3(64 * NS_ * CG_), P->lds_colfast,
                              st, P->kt_ev[2 * n], P->kt_ev[2 * n + 1], 0, g, in, out, P->ST, P->theta, P->tw2,
                              P->twM, P->Khat, use_reg, pc, P->prow);
    } else {
        hipLaunchKernelGGL((k_col_fast<M_, L_, NS_, CG_, KF32>), dim3(g.n1), dim3(64 * NS_ * CG_), P->lds_colfast, st,
                           g, in, out, P->ST, P->theta, P->tw2, P->twM, P->Khat, use_reg, pc, P->prow);
    }
}
template <int M_, int L_, int NS_ = 4, int CG_ = 2>
void launch_colfast(smsm_plan* P, const double2* in, double2* out, int use_reg, const ColCg& pc, hipStream_t st) {
    // the complex64 table only matters where the regulariser term is applied
    if (use_reg && P->khat_f32) launch_colfast_k<M_, L_, NS_, CG_, true>(P, in, out, use_reg, pc, st);
    else launch_colfast_k<M_, L_, NS_, CG_, false>(P, in, out, use_reg, pc, st);
}

// Column pass (hybrid in -> hybrid out).  For MODE == COL_NORMAL, `pc` may
// ask for the fused CG direction update: the input is then pc.p, rebuilt from
// pc.r, and Re <p, out> partials go to pc.pq (P->npc of them).
template <int MODE>
smsm_status col(smsm_plan* P, const double2* in, double2* out, int use_reg, const ColCg& pc, hipStream_t st) {
    const Geo& g = P->g;
    if (MODE == COL_NORMAL && P->col_fast >= 0) {
        switch (P->col_fast) {
            case 0: launch_colfast<16, 2>(P, in, out, use_reg, pc, st); break;
            case 1: launch_colfast<16, 3>(P, in, out, use_reg, pc, st); break;
            case 2: launch_colfast<32, 2>(P, in, out, use_reg, pc, st); break;
            case 3: launch_colfast<32, 3>(P, in, out, use_reg, pc, st); break;
            case 4: launch_colfast<64, 2>(P, in, out, use_reg, pc, st); break;
            case 5: launch_colfast<64, 3>(P, in, out, use_reg, pc, st); break;
            case 6: launch_colfast<32, 2, 8, 1>(P, in, out, use_reg, pc, st); break;
            case 7: launch_colfast<16, 2, 8, 1>(P, in, out, use_reg, pc, st); break;
            case 8: launch_colfast<128, 2, 2, 4>(P, in, out, use_reg, pc, st); break;
            case 9: launch_colfast<128, 3, 2, 4>(P, in, out, use_reg, pc, st); break;
            case 10: launch_colfast<64, 2, 2, 4>(P, in, out, use_reg, pc, st); break;
            default: launch_colfast<64, 3, 2, 4>(P, in, out, use_reg, pc, st); break;
        }
        LAUNCH_CHECK();
        return SMSM_OK;
    }
    const long nvec = (long)g.B * g.n1 * g.n2;
    // the odd-length pass takes the direction update and the Re <p, out> partials itself
    const bool fused = MODE == COL_NORMAL && P->col_mix >= 0;
    if (pc.mode != 0 && !fused) {
        hipLaunchKernelGGL(k_hyb_pupdate, vec_grid(), dim3(kThreads), 0, st, nvec, pc.r, pc.p_old, pc.p, pc.x,
                           pc.alpha_prev, pc.rr_new, pc.nrr, pc.rr_old, pc.rr_out, pc.mode == 1 ? 1 : 0);
        LAUNCH_CHECK();
        in = pc.p;
    }
    if (fused) {
#define COLMIX_LAUNCH(M_, L_, NS_, CG_)                                                                          \
    hipLaunchKernelGGL((k_col_mix<M_, L_, NS_, CG_>), dim3(g.n1), dim3(64 * NS_ * CG_), P->lds_colmix, st, g, in, \
                       out, P->ST, P->theta, P->tau, P->tw2, P->twM, P->Khat, use_reg, pc)
        switch (P->col_mix) {
            case 0: COLMIX_LAUNCH(56, 3, 4, 2); break;
            case 1: COLMIX_LAUNCH(56, 2, 4, 2); break;
            case 2: COLMIX_LAUNCH(48, 3, 4, 2); break;
            case 3: COLMIX_LAUNCH(48, 2, 4, 2); break;
            case 4: COLMIX_LAUNCH(28, 2, 8, 1); break;
            case 5: COLMIX_LAUNCH(24, 2, 8, 1); break;
            case 6: COLMIX_LAUNCH(28, 2, 4, 2); break;
            case 7: COLMIX_LAUNCH(112, 2, 2, 4); break;
            case 8: COLMIX_LAUNCH(96, 3, 2, 4); break;
            case 9: COLMIX_LAUNCH(96, 2, 2, 4); break;
            default: COLMIX_LAUNCH(112, 3, 2, 4); break;
        }
#undef COLMIX_LAUNCH
    } else {
        hipLaunchKernelGGL(k_col<MODE>, dim3(g.n1), dim3(kColThreads), P->lds_col, st, g, in, out,
                           P->ST, P->theta, P->tau, P->tw2, P->twM, P->tw1, P->Kc, use_reg, P->ytil);
    }
    LAUNCH_CHECK();
    if (pc.mode != 0 && !fused) {
        hipLaunchKernelGGL(k_hyb_dot, vec_grid(), dim3(kThreads), 0, st, nvec, pc.p, out, pc.pq);
        LAUNCH_CHECK();
    }
    return SMSM_OK;
}

ColCg no_cg() {
    ColCg c{};
    c.mode = 0;
    return c;
}

// Natural band columns of the hybrid vector `in` (pcol), and its transposed
// band rows (prow) unless the fast column pass already wrote them.
smsm_status band_extract(smsm_plan* P, const double2* in, bool write_prow, hipStream_t st) {
    const Geo& g = P->g;
    hipLaunchKernelGGL(k_band_extract, dim3((g.n2 / 16) * (P->np_band / 16), g.B), dim3(64 * EXTRACT_WAVES), 0, st,
                       g.n1,
                       g.n2, g.e, P->np_band, in, P->fx, P->pcol, P->prow, write_prow ? 1 : 0);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// Band corrections of the vector whose band copies band_extract made last;
// Re <p, correction> partials to P->bpart.
smsm_status band_corr(smsm_plan* P, hipStream_t st) {
    const Geo& g = P->g;
    BandArgs a{};
    a.g = g;
    a.pcol = P->pcol;
    a.prow = P->prow;
    a.Dside = P->Dside;
    a.Dhat = P->Dhat;
    a.Dx = P->Dx;
    a.crow = P->crow;
    a.ccol = P->ccol;
    a.ccorner = P->ccorner;
    a.part = P->bpart;
    void* args[] = {&a};
    if (hipLaunchKernel((const void*)(P->khat_f32 ? P->band_f32 : P->band), dim3(band_items(g), g.L), dim3(64 * g.Ns),
                        args, P->lds_band, st) !=
        hipSuccess)
        return SMSM_E_DEVICE;
    LAUNCH_CHECK();
    return SMSM_OK;
}

template <int MODE, bool WU, bool BAND>
const void* hyb_update_fn_x(int xw) {
    switch (xw) {
        case 1: return (const void*)&k_hyb_update<MODE, 1, WU, BAND>;
        case 2: return (const void*)&k_hyb_update<MODE, 2, WU, BAND>;
        case 4: return (const void*)&k_hyb_update<MODE, 4, WU, BAND>;
        default: return nullptr;
    }
}
template <int MODE>
const void* hyb_update_fn_m(int xw, bool wu, bool band) {
    if (wu) return band ? hyb_update_fn_x<MODE, true, true>(xw) : hyb_update_fn_x<MODE, true, false>(xw);
    return band ? hyb_update_fn_x<MODE, false, true>(xw) : hyb_update_fn_x<MODE, false, false>(xw);
}
const void* hyb_update_fn(int mode, int xw, bool wu, bool band) {
    switch (mode) {
        case 0: return hyb_update_fn_m<0>(xw, wu, band);
        case 1: return hyb_update_fn_m<1>(xw, wu, band);
        default: return hyb_update_fn_m<2>(xw, wu, band);
    }
}

// Hybrid vector pass (see k_hyb_update).
smsm_status hyb_update(smsm_plan* P, HybArgs a, hipStream_t st) {
    a.g = P->g;
    a.bi = BandInj{P->crow, P->ccol, P->ccorner, P->finv, band_ds(P->g.Ns, P->g.nc)};
    a.pq = P->pq;
    a.npq = P->npc + (a.use_band ? band_items(P->g) * P->g.L : 0);
    if (!a.alpha_out) a.alpha_out = P->cgs + 8;
    a.flags = P->flags;
    const void* fn = hyb_update_fn(a.mode, P->hyb_xw, hyb_ly(P->g) == 64, a.use_band != 0);
    void* args[] = {&a};
    if (!fn || hipLaunchKernel(fn, P->hyb_grid, dim3(64 * HYB_WAVES), args, 0, st) != hipSuccess) return SMSM_E_DEVICE;
    LAUNCH_CHECK();
    return SMSM_OK;
}

// x += alpha p with the last step length (cgs + 8): the last CG step of a cycle.
smsm_status x_step(smsm_plan* P, hipStream_t st) {
    const long nvec = (long)P->g.B * P->g.n1 * P->g.n2;
    hipLaunchKernelGGL(k_x_step, vec_grid(), dim3(kThreads), 0, st, nvec, P->x, P->p, P->cgs + 8);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// Hybrid q = column pass + band correction of the hybrid vector `in`, then the
// vector pass `a` (mode 0 or 1).
smsm_status hyb_apply(smsm_plan* P, const double2* in, int mode_col, bool reg, HybArgs a, hipStream_t st) {
    smsm_status s = mode_col == COL_REG ? col<COL_REG>(P, in, P->h2, 1, no_cg(), st)
                                        : col<COL_NORMAL>(P, in, P->h2, reg ? 1 : 0, no_cg(), st);
    if (s) return s;
    if (reg) {
        if ((s = band_extract(P, in, !(mode_col == COL_NORMAL && P->col_fast >= 0), st))) return s;
        if ((s = band_corr(P, st))) return s;
    }
    a.h2 = P->h2;
    a.use_band = reg ? 1 : 0;
    return hyb_update(P, a, st);
}

smsm_status band_tables(smsm_plan* P, hipStream_t st) {
    const Geo& g = P->g;
    const long total = (long)g.L * (4 * g.e + 4 * g.e * g.e + 1) * g.Ns * g.Ns * g.nc * g.nc;
    const int blocks = (int)std::min<long>(8192, (total + kThreads - 1) / kThreads);
    // the format every reader of these tables follows until the next build
    P->khat_f32 = (P->prm.flags & SMSM_FLAG_REG_F32) != 0;
    hipLaunchKernelGGL(k_band_tables, dim3(blocks), dim3(kThreads), 0, st, g, P->W, 0.5 * P->prm.lambda,
                       P->Kc, P->Dside, P->Dx, P->khat_f32 ? 1 : 0);
    LAUNCH_CHECK();
    if (is_pow2(g.n1))
        hipLaunchKernelGGL(k_band_rowhat<true>, dim3(g.L * 2 * g.e * g.Ns * g.nc), dim3(kThreads), 0, st, g,
                           P->Dside, P->tw1, P->Dhat, P->khat_f32 ? 1 : 0);
    else
        hipLaunchKernelGGL(k_band_rowhat<false>, dim3(g.L * 2 * g.e * g.Ns * g.nc), dim3(kThreads), 0, st, g,
                           P->Dside, P->tw1, P->Dhat, P->khat_f32 ? 1 : 0);
    LAUNCH_CHECK();
    if (P->col_mix >= 0) {
        // the odd-length pass's per-column tap table lives in the (otherwise unused) Khat region
        hipLaunchKernelGGL(k_colmix_taps, dim3(g.n1), dim3(256), 0, st, g, P->Kc, P->tw1, P->Khat);
        LAUNCH_CHECK();
    }
    if (P->col_fast >= 0) {
        hipLaunchKernelGGL(k_hankel_image, dim3(g.n1, g.L * g.Ns * (g.Ns + 1) / 2), dim3(kThreads), 0, st, g, P->Kc, P->tw1,
                           P->tw2, P->Khat, P->khat_f32 ? 1 : 0);
        LAUNCH_CHECK();
    }
    P->have_weights = true;
    return SMSM_OK;
}

// A^H y (y c64) in the hybrid layout into `out`.
smsm_status chain_AH_hyb(smsm_plan* P, const float2* y, double2* out, hipStream_t st) {
    const Geo& g = P->g;
    hipLaunchKernelGGL(k_yrows_inv, dim3(g.M / P->TRy, g.Ns * g.Nc), dim3(kThreads), P->lds_rows, st, g, y,
                       P->ytil, P->tw1, P->TRy);
    LAUNCH_CHECK();
    return col<COL_ADJ>(P, nullptr, out, 0, no_cg(), st);
}

// out = N(v) (mode_col COL_NORMAL, reg), (lambda/2) sum H^H(H W) (COL_REG) or
// A^H A v (COL_NORMAL, !reg); natural in and out.
smsm_status chain_normal(smsm_plan* P, const double2* v, double2* out, int mode_col, bool reg, hipStream_t st) {
    smsm_status s = rows_inv(P, v, P->h1, st);
    if (s) return s;
    HybArgs a{};
    a.mode = 0;
    a.out = P->q;
    if ((s = hyb_apply(P, P->h1, mode_col, reg, a, st))) return s;
    return rows_fwd(P, P->q, out, st);
}

// G = Gram of the natural vector v; vh is its hybrid form, or null to compute it.
smsm_status chain_gram(smsm_plan* P, const double2* v, const double2* vh, double2* G, hipStream_t st) {
    const Geo& g = P->g;
    smsm_status s = SMSM_OK;
    if (P->prm.flags & SMSM_FLAG_GRAM_BF16) {
        // the GEMM form on the BF16 matrix cores (needs the natural v only)
        const AlGeo a = anchor_geo(g);
        const int nch = gram_bf16_chunks(a);
        hipLaunchKernelGGL(k_gram_bf16, dim3(a.KB * (a.KB + 1) / 2, nch, g.L), dim3(kThreads), 0, st, a, v,
                           P->gbpart);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_gram_bf16_sum, dim3(kPadBlocks, g.L), dim3(kThreads), 0, st, a, P->gbpart, nch, G);
        LAUNCH_CHECK();
        return SMSM_OK;
    }
    if (!vh) {
        if ((s = rows_inv(P, v, P->h1, st))) return s;
        vh = P->h1;
    }
    const size_t lds = P->lds_gram;
    if (!is_pow2(g.n2)) {
        hipLaunchKernelGGL(k_gram_q_any, dim3(g.n1), dim3(512), lds, st, g, vh, P->tw2, P->gpart);
    } else switch (g.n2) {
        case 16: hipLaunchKernelGGL(k_gram_q<16>, dim3(g.n1), dim3(kThreads), lds, st, g, vh, P->tw2, P->gpart); break;
        case 32: hipLaunchKernelGGL(k_gram_q<32>, dim3(g.n1), dim3(kThreads), lds, st, g, vh, P->tw2, P->gpart); break;
        case 64: hipLaunchKernelGGL(k_gram_q<64>, dim3(g.n1), dim3(kThreads), lds, st, g, vh, P->tw2, P->gpart); break;
        case 128: hipLaunchKernelGGL(k_gram_q<128>, dim3(g.n1), dim3(kThreads), lds, st, g, vh, P->tw2, P->gpart); break;
        default: hipLaunchKernelGGL(k_gram_q<256>, dim3(g.n1), dim3(kThreads), lds, st, g, vh, P->tw2, P->gpart); break;
    }
    LAUNCH_CHECK();
    const int wpb = kThreads / 64;
    const int nwc = g.L * g.npairs * g.nc;
    if (is_pow2(g.n1))
        hipLaunchKernelGGL(k_gram_c<true>, dim3((nwc + wpb - 1) / wpb), dim3(kThreads), 0, st, g, P->gpart, P->tw1,
                           P->gC);
    else
        hipLaunchKernelGGL(k_gram_c<false>, dim3((nwc + wpb - 1) / wpb), dim3(kThreads), 0, st, g, P->gpart, P->tw1,
                           P->gC);
    LAUNCH_CHECK();
    // natural band columns of v (contiguous in ky) for the column sums
    if ((s = band_extract(P, vh, false, st))) return s;
    const bool p2 = is_pow2(g.n1) && is_pow2(g.n2);
    const dim3 gl(2 * g.e * g.L * g.npairs, 2);
    if (p2)
        hipLaunchKernelGGL(k_gram_lines<true>, gl, dim3(kThreads), P->lds_gram_lines, st, g, v, P->pcol, P->grow,
                           P->gcol);
    else
        hipLaunchKernelGGL(k_gram_lines<false>, gl, dim3(kThreads), P->lds_gram_lines, st, g, v, P->pcol, P->grow,
                           P->gcol);
    LAUNCH_CHECK();
    const long ncor = (long)nwc * g.nc * 4 * g.e * g.e;
    const dim3 gcg((int)std::min<long>(4096, (ncor + kThreads - 1) / kThreads));
    if (p2)
        hipLaunchKernelGGL(k_gram_corners<true>, gcg, dim3(kThreads), 0, st, g, v, P->gcor);
    else
        hipLaunchKernelGGL(k_gram_corners<false>, gcg, dim3(kThreads), 0, st, g, v, P->gcor);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gram_assemble, dim3(nwc * g.nc), dim3(64), 0, st, g, P->gC, P->grow, P->gcol, P->gcor, G);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// W = (G + eps I)^(-1/2) with eps_l = mult * src[l] (device array).
smsm_status chain_weights(smsm_plan* P, const double2* G, const double* src, double mult, hipStream_t st) {
    const Geo& g = P->g;
    const int nit = P->ns_iters, KP = P->KP;
    hipLaunchKernelGGL(k_dense_pad, dim3(kPadBlocks, g.L), dim3(kThreads), 0, st, g.K, KP, G, src, mult, P->Y0,
                       P->part0);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ns_start, dim3(kPadBlocks, g.L), dim3(kThreads), 0, st, g.K, KP, g.L, src, mult,
                       P->part0, kPadBlocks, P->Y0, P->Z0, P->wscale, P->done, nit, P->nsmu);
    LAUNCH_CHECK();
    double2* Y[2] = {P->Y0, P->Y1};
    double2* Z[2] = {P->Z0, P->Z1};
    for (int k = 0; k < nit; ++k) {
        const int a = k & 1, bsel = a ^ 1;
        HgArgs t{};
        t.A0 = Z[a]; t.B0 = Y[a]; t.C0 = P->T;
        t.done_cur = P->done + (size_t)k * g.L;
        t.part_out = P->part0;
        t.mu = P->nsmu + (size_t)k * g.L;
        t.mu_stride = 1;
        hipLaunchKernelGGL(k_zgemm<HG_NS>, dim3(P->ntile, 1, g.L), dim3(64 * HW), 0, st, g.K, KP, t);
        LAUNCH_CHECK();
        HgArgs u{};
        u.A0 = Y[a]; u.B0 = P->T; u.C0 = Y[bsel];
        u.A1 = P->T; u.B1 = Z[a]; u.C1 = Z[bsel];
        u.done_cur = P->done + (size_t)k * g.L;
        u.done_next = P->done + (size_t)(k + 1) * g.L;
        u.last = P->done + (size_t)(nit + 1) * g.L;
        u.par = bsel;
        u.tol2 = kNsTol * kNsTol;
        u.part_in = P->part0;
        u.np_in = P->ntile;
        hipLaunchKernelGGL(k_zgemm<HG_PAIR>, dim3(P->ntile, 1, 2 * g.L), dim3(64 * HW), 0, st, g.K, KP, u);
        LAUNCH_CHECK();
    }
    const long tot = (long)g.L * g.K * g.K;
    hipLaunchKernelGGL(k_ns_finish, dim3((int)((tot + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, g.K,
                       KP, g.L, P->Z0, P->Z1, P->done + (size_t)(nit + 1) * g.L, P->done + (size_t)nit * g.L,
                       P->wscale, P->W, P->flags);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// lmax[l] = largest eigenvalue of G_l by repeated normalised squaring
// P <- P^2 / ||P||_F^2 and the Rayleigh quotient tr(G P) / tr(P).
smsm_status chain_lmax(smsm_plan* P, const double2* G, double* lmax, hipStream_t st) {
    const Geo& g = P->g;
    const int KP = P->KP;
    hipLaunchKernelGGL(k_dense_pad, dim3(kPadBlocks, g.L), dim3(kThreads), 0, st, g.K, KP, G, nullptr, 0.0, P->T,
                       P->part0);
    LAUNCH_CHECK();
    const double2* cur = P->T;
    double2* buf[2] = {P->Y0, P->Y1};
    double* part[2] = {P->part0, P->part1};
    for (int k = 0; k < kSqSteps; ++k) {
        HgArgs a{};
        a.A0 = cur; a.B0 = cur; a.C0 = buf[k & 1];
        a.part_in = part[k & 1];
        a.np_in = k == 0 ? kPadBlocks : P->ntile;
        a.part_out = part[(k + 1) & 1];
        hipLaunchKernelGGL(k_zgemm<HG_NORM>, dim3(P->ntile, 1, g.L), dim3(64 * HW), 0, st, g.K, KP, a);
        LAUNCH_CHECK();
        cur = buf[k & 1];
    }
    hipLaunchKernelGGL(k_trace_part, dim3(kPadBlocks, g.L), dim3(kThreads), 0, st, g.K, KP, G, cur, P->part0);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_trace_final, dim3(g.L), dim3(kThreads), 0, st, g.L, P->part0, kPadBlocks, lmax);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// Point the plan's scratch buffers into the workspace at `base` (null: none).
void bind_workspace(smsm_plan* P, void* base) {
    P->ws = base;
    char* c = static_cast<char*>(base);
    const WsLayout& w = P->wo;
    auto d2 = [&](size_t o) { return c ? (double2*)(c + o) : nullptr; };
    auto d1 = [&](size_t o) { return c ? (double*)(c + o) : nullptr; };
    P->x = d2(w.x); P->b = d2(w.b); P->r = d2(w.r); P->p = d2(w.p); P->q = d2(w.q);
    P->h1 = d2(w.h1); P->h2 = d2(w.h2); P->ytil = d2(w.ytil);
    P->G = d2(w.G); P->W = d2(w.W); P->Y0 = d2(w.Y0); P->Y1 = d2(w.Y1);
    P->Z0 = d2(w.Z0); P->Z1 = d2(w.Z1); P->T = d2(w.T);
    P->Kc = d2(w.Kc); P->Khat = d2(w.Khat); P->Dside = d2(w.Dside); P->Dx = d2(w.Dx);
    P->crow = d2(w.crow); P->ccol = d2(w.ccol); P->ccorner = d2(w.ccorner); P->Dhat = d2(w.Dhat);
    P->pcol = d2(w.pcol); P->prow = d2(w.prow);
    P->gpart = d2(w.gpart); P->gC = d2(w.gC); P->grow = d2(w.grow); P->gcol = d2(w.gcol); P->gcor = d2(w.gcor);
    P->pr = d1(w.pr); P->pq = d1(w.pq); P->part0 = d1(w.part0); P->part1 = d1(w.part1);
    P->bpart = c ? P->pq + P->npc : nullptr;   // band partials follow the column-pass partials
    P->sigma = d1(w.sigma); P->eps = d1(w.eps); P->wscale = d1(w.wscale); P->epsin = d1(w.epsin);
    P->nsmu = d1(w.nsmu);
    P->done = c ? (int*)(c + w.done) : nullptr;
    P->cgs = d1(w.cgs);
    P->gbpart = P->gram_bf16_ws ? d2(w.gbpart) : nullptr;
    // the weight tables of an earlier workspace are not in this one
    P->have_weights = false;
}

// Entry points that run kernels on the plan's scratch need a bound workspace.
smsm_status ready(smsm_plan* P) {
    if (!P || !P->ws) return SMSM_E_INVALID;
    return hipSetDevice(P->dev) == hipSuccess ? SMSM_OK : SMSM_E_DEVICE;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

extern "C" {

const char* smsm_status_string(smsm_status s) {
    switch (s) {
        case SMSM_OK: return "ok";
        case SMSM_E_INVALID: return "invalid argument";
        case SMSM_E_UNSUPPORTED: return "unsupported geometry or sampling pattern";
        case SMSM_E_NOMEM: return "device allocation failed";
        case SMSM_E_DEVICE: return "HIP runtime error";
        case SMSM_E_NUMERIC: return "non-finite or non-positive CG curvature";
        case SMSM_E_NOT_CONVERGED: return "weights iteration did not converge within ns_max_iter";
        case SMSM_E_SCRATCH: return "workspace larger than the static scratch of smsm_solve_noalloc";
    }
    return "unknown status";
}

smsm_status smsm_plan_create(const smsm_geometry* geom, const smsm_params* params, const void* coil_maps_dev,
                             const uint8_t* shot_mask, const double* caipi_shift, void* stream,
                             smsm_plan** out) {
    if (!out) return SMSM_E_INVALID;
    *out = nullptr;
    if (!geom || !coil_maps_dev || !shot_mask) return SMSM_E_INVALID;
    smsm_status ps = check_params(params);
    if (ps) return ps;
    const int n1 = geom->n1, n2 = geom->n2, L = geom->n_slices, Ns = geom->n_shots, Nc = geom->n_coils,
              r = geom->filt;
    if (n1 <= 0 || n2 <= 0 || L <= 0 || Ns <= 0 || Nc <= 0 || r <= 0) return SMSM_E_INVALID;
    if (!length_ok(n1) || !length_ok(n2)) return SMSM_E_UNSUPPORTED;
    if (!is_pow2(Ns) || Ns > 8 || n2 / Ns < 8 || L > 4) return SMSM_E_UNSUPPORTED;
    if (r < 2 || 2 * r - 1 > std::min(n1, n2) / 2 || Ns * r * r > 256 || 2 * r - 1 > BAND_MAX_NC)
        return SMSM_E_UNSUPPORTED;
    // interleaved sampling of Eq. 2 only
    for (int i = 0; i < Ns; ++i)
        for (int j = 0; j < n2; ++j)
            if ((shot_mask[i * n2 + j] != 0) != (j % Ns == i)) return SMSM_E_UNSUPPORTED;

    smsm_plan* P = new (std::nothrow) smsm_plan();
    if (!P) return SMSM_E_NOMEM;
    if (hipGetDevice(&P->dev) != hipSuccess) { delete P; return SMSM_E_DEVICE; }
    Geo& g = P->g;
    g.n1 = n1; g.n2 = n2; g.L = L; g.Ns = Ns; g.Nc = Nc; g.r = r;
    g.K = Ns * r * r; g.nc = 2 * r - 1; g.e = r - 1; g.M = n2 / Ns;
    g.logn1 = pow2_log(n1); g.logn2 = pow2_log(n2); g.logM = pow2_log(g.M);
    g.B = L * Ns;
    g.nband = 2 * g.e * n1 + 2 * g.e * (n2 - 2 * g.e);
    g.npairs = Ns * (Ns + 1) / 2;
    P->prm = *params;
    P->ns_iters = params->ns_max_iter > 0 ? params->ns_max_iter : kNsDefaultIters;

    P->TR = std::max(1, std::min(n2, 2048 / n1));
    while (P->TR & (P->TR - 1)) P->TR &= P->TR - 1;   // a power of two
    P->TRy = std::min(g.M & -g.M, P->TR);              // divides the M folded lines
    P->lds_rows = (size_t)P->TR * (n1 + 1) * sizeof(double2) + 16 * sizeof(double);
    int max_lds = 0;
    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->dev);
    if (max_lds <= 0) max_lds = 65536;
    // the generic column pass: its coil loop accumulates in registers (B n2 <=
    // KCOL_ACC x threads; a larger accumulator would not fit its shared memory
    // either); coils per pass, the most (4, 2, 1) its shared memory holds with
    // the transform of a pass (cb B sequences of M) within the outputs the
    // loop's mixed-length transforms keep in registers
    if (g.B * n2 > KCOL_ACC * kColThreads) {
        delete P;
        return SMSM_E_UNSUPPORTED;
    }
    g.cb = 4;
    while (g.cb > 1 && ((size_t)col_lds(g).total * sizeof(double2) > (size_t)max_lds ||
                        g.cb * g.B * g.M > KCOL_FOUT * kColThreads))
        g.cb >>= 1;
    P->lds_col = (size_t)col_lds(g).total * sizeof(double2);
    P->lds_gram = (size_t)(g.B * n2 + n2) * sizeof(double2);
    P->lds_gram_lines = (size_t)(1 + g.nc) * std::max(n1, n2) * sizeof(double2);
    set_rows_shape(P, (n1 == 16) ? 16 : (n1 == 32 ? 8 : 4));
    if (!set_hyb_shape(P, 4) && !set_hyb_shape(P, 2) && !set_hyb_shape(P, 1)) {
        delete P;                                   // n1 < HYB_WAVES (64 / min(n2, 64))
        return SMSM_E_UNSUPPORTED;
    }
    P->npr_max = hyb_blocks(g, 1);                  // the |r|^2 ring is sized for every shape
    P->np_band = 16 * ((4 * g.e + 15) / 16);
    P->KP = dense_stride(g.K);
    P->ntile = dense_tiles(g.K);
    P->npmax = std::max(P->ntile, 2 * kPadBlocks);
    P->lds_band = band_lds_bytes(g);
    P->band = band_fn(g.nc, Ns);
    P->band_f32 = band_fn(g.nc, Ns, true);
    if (!P->band) {
        delete P;
        return SMSM_E_UNSUPPORTED;
    }
    P->lds_colfast = (size_t)colfast_lds_total(g) * sizeof(double2);
    if (P->lds_col > (size_t)max_lds || P->lds_gram > (size_t)max_lds || P->lds_gram_lines > (size_t)max_lds ||
        P->lds_band + 16 * sizeof(double) > (size_t)max_lds) {
        delete P;
        return SMSM_E_UNSUPPORTED;
    }
    for (int k = 0; k < (int)(sizeof(kColFast) / sizeof(kColFast[0])); ++k)
        if (kColFast[k].M == g.M && kColFast[k].L == L && kColFast[k].Ns == Ns && is_pow2(n1) && is_pow2(n2) &&
            P->lds_colfast <= (size_t)max_lds)
            P->col_fast = k;
    if (P->col_fast < 0)
        for (int k = 0; k < (int)(sizeof(kColMix) / sizeof(kColMix[0])); ++k) {
            const ColMixInst& c = kColMix[k];
            const size_t bytes = (size_t)colmix_lds_total(g, colmix_wb(c.M, c.L, c.Ns, c.CG)) * sizeof(double2);
            const bool taps_fit = (size_t)n1 * L * Ns * Ns * g.nc <= (size_t)L * Ns * (Ns + 1) / 2 * n1 * n2;
            if (c.M == g.M && c.L == L && c.Ns == Ns && 64 * c.Ns * c.CG == kColThreads && bytes <= (size_t)max_lds &&
                taps_fit) {
                P->col_mix = k;
                P->lds_colmix = bytes;
            }
        }

    // device memory: the plan arena holds what creation derives; every buffer
    // a solve or operator chain writes lives in the caller's workspace
    const size_t nvec = (size_t)L * Ns * n2 * n1;
    const size_t KK = (size_t)L * g.K * g.K;
    const size_t KKP = (size_t)L * P->KP * P->KP;
    const size_t ntab = (size_t)L * 4 * g.e * Ns * Ns * g.nc * g.nc;
    const size_t nds = band_ds(Ns, g.nc);
    const size_t nper = (size_t)L * g.npairs * g.nc * g.nc;
    Carver cv;
    const size_t oST = cv.take<double2>((size_t)L * Nc * n1 * n2);
    const size_t otw1 = cv.take<double2>(n1), otw2 = cv.take<double2>(n2), otwM = cv.take<double2>(g.M);
    const size_t oth = cv.take<double2>((size_t)L * n2), otau = cv.take<double2>((size_t)Ns * n2);
    const size_t ofx = cv.take<double2>((size_t)n1 * P->np_band), ofinv = cv.take<double2>((size_t)n1 * HYB_MAX_E2);
    const size_t oflags = cv.take<int>(4);
    P->npc = (P->col_fast >= 0 || P->col_mix >= 0) ? n1 : kVecBlocks;
    Carver wv;
    WsLayout& w = P->wo;
    w.x = wv.take<double2>(nvec); w.b = wv.take<double2>(nvec); w.r = wv.take<double2>(nvec);
    w.p = wv.take<double2>(nvec); w.q = wv.take<double2>(nvec);
    w.h1 = wv.take<double2>(nvec); w.h2 = wv.take<double2>(nvec);
    w.ytil = wv.take<double2>((size_t)Ns * Nc * n1 * g.M);
    w.G = wv.take<double2>(KK); w.W = wv.take<double2>(KK);
    w.Y0 = wv.take<double2>(KKP); w.Y1 = wv.take<double2>(KKP);
    w.Z0 = wv.take<double2>(KKP); w.Z1 = wv.take<double2>(KKP); w.T = wv.take<double2>(KKP);
    w.Kc = wv.take<double2>((size_t)L * Ns * Ns * g.nc * g.nc);
    w.Khat = wv.take<double2>((size_t)L * Ns * (Ns + 1) / 2 * n1 * n2);   // Hermitian pairs j <= i
    w.Dside = wv.take<double2>(ntab);
    w.Dx = wv.take<double2>(ntab * g.e);
    w.crow = wv.take<double2>((size_t)g.B * 2 * g.e * n1);
    w.ccol = wv.take<double2>(nds * g.B * 2 * g.e * n2);
    w.ccorner = wv.take<double2>((size_t)g.B * 4 * g.e * g.e);
    w.Dhat = wv.take<double2>((size_t)L * 2 * g.e * Ns * g.nc * Ns * n1);
    w.pcol = wv.take<double2>((size_t)g.B * 4 * g.e * n2);
    w.prow = wv.take<double2>((size_t)g.B * 4 * g.e * n1);
    w.gpart = wv.take<double2>((size_t)L * g.npairs * n1 * g.nc); w.gC = wv.take<double2>(nper);
    w.grow = wv.take<double2>(nper * 2 * g.e); w.gcol = wv.take<double2>(nper * 2 * g.e);
    w.gcor = wv.take<double2>(nper * 4 * g.e * g.e);
    // partial sums: |r|^2 ring [3][npr]; Re <p, N p> [npc column pass | band]
    w.pr = wv.take<double>(3 * (size_t)P->npr_max);
    w.pq = wv.take<double>((size_t)P->npc + (size_t)band_items(g) * L);
    w.part0 = wv.take<double>((size_t)L * P->npmax); w.part1 = wv.take<double>((size_t)L * P->npmax);
    w.sigma = wv.take<double>(L); w.eps = wv.take<double>(L); w.wscale = wv.take<double>(L);
    w.epsin = wv.take<double>(L); w.nsmu = wv.take<double>((size_t)P->ns_iters * L);
    w.done = wv.take<int>((size_t)(P->ns_iters + 2) * L);
    w.cgs = wv.take<double>(16);
    P->gram_bf16_ws = (params->flags & SMSM_FLAG_GRAM_BF16) != 0;
    if (P->gram_bf16_ws) {   // chunk partials of the GEMM-form Gram, only for plans created with it
        const AlGeo a = anchor_geo(g);
        w.gbpart = wv.take<double2>((size_t)L * gram_bf16_chunks(a) * (a.KB * (a.KB + 1) / 2) * 64 * 64);
    }
    P->ws_bytes = (wv.off + 255) & ~size_t(255);

    P->bytes = cv.off;
    if (hipMalloc(&P->arena, P->bytes) != hipSuccess) { delete P; return SMSM_E_NOMEM; }
    char* base = static_cast<char*>(P->arena);
    P->ST = (double2*)(base + oST);
    P->tw1 = (double2*)(base + otw1); P->tw2 = (double2*)(base + otw2); P->twM = (double2*)(base + otwM);
    P->theta = (double2*)(base + oth); P->tau = (double2*)(base + otau);
    P->fx = (double2*)(base + ofx); P->finv = (double2*)(base + ofinv);
    P->flags = (int*)(base + oflags);

    // host tables: twiddles, CAIPI phases, shot modulation
    std::vector<double2> t1, t2, tM, th((size_t)L * n2), ta((size_t)Ns * n2);
    twiddles(n1, t1);
    twiddles(n2, t2);
    twiddles(g.M, tM);
    for (int l = 0; l < L; ++l) {
        const double s = caipi_shift ? caipi_shift[l] : (double)l / (double)L;
        for (int j = 0; j < n2; ++j) {
            const long double v = (long double)s * (long double)(j - n2 / 2);
            const long double fr = v - floorl(v);
            const long double a = -2.0L * 3.14159265358979323846264338327950288L * fr;
            th[(size_t)l * n2 + j] = make_double2((double)cosl(a), (double)sinl(a));
        }
    }
    for (int i = 0; i < Ns; ++i)
        for (int n = 0; n < n2; ++n) {
            const double2 w = t2[(size_t)(i * n) % n2];
            const double sg = (n & 1) ? -1.0 : 1.0;
            ta[(size_t)i * n2 + n] = make_double2(sg * w.x, sg * w.y);
        }
    // kx transforms restricted to the band columns (see k_band_extract, BandInj)
    const int e2 = 2 * g.e, npb = P->np_band;
    std::vector<double2> fxh((size_t)n1 * npb, make_double2(0.0, 0.0)), fih((size_t)n1 * HYB_MAX_E2, make_double2(0.0, 0.0));
    {
        const long double pi2 = 2.0L * 3.14159265358979323846264338327950288L;
        const long double isq = 1.0L / sqrtl((long double)n1);
        auto phase = [&](int kx, int x) {   // e^{-2 pi i (kx - n1/2)(x - n1/2)/n1}, argument reduced exactly
            const long long t = (long long)(kx - n1 / 2) * (long long)(x - n1 / 2);
            const long long m = ((t % n1) + n1) % n1;
            const long double a = -pi2 * (long double)m / (long double)n1;
            return make_double2((double)(cosl(a) * isq), (double)(sinl(a) * isq));
        };
        for (int x = 0; x < n1; ++x) {
            for (int c = 0; c < 2 * e2; ++c) fxh[(size_t)x * npb + c] = phase(c < e2 ? c : n1 - 2 * e2 + c, x);
            for (int c = 0; c < e2; ++c) {
                const double2 v = phase(c < g.e ? c : n1 - e2 + c, x);
                fih[(size_t)x * HYB_MAX_E2 + c] = make_double2(v.x, -v.y);
            }
        }
    }
    hipStream_t st = S(stream);
    bool ok = hipMemcpyAsync(P->fx, fxh.data(), fxh.size() * sizeof(double2), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(P->finv, fih.data(), fih.size() * sizeof(double2), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(P->tw1, t1.data(), n1 * sizeof(double2), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(P->tw2, t2.data(), n2 * sizeof(double2), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(P->twM, tM.data(), g.M * sizeof(double2), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(P->theta, th.data(), th.size() * sizeof(double2), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(P->tau, ta.data(), ta.size() * sizeof(double2), hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_transpose_coils, dim3(2048), dim3(kThreads), 0, st, n1, n2, (long)L * Nc,
                           (const float2*)coil_maps_dev, P->ST);
        ok = hipGetLastError() == hipSuccess;
    }
    if (ok) {
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(kThreads), 0, st, 4L, P->flags);

        ok = hipGetLastError() == hipSuccess;
    }
    // shared-memory opt-in: each kernel's cap is the dynamic size it is launched
    // with (static shared memory counts against the same per-block limit)
    if (ok) {
        struct Opt { const void* f; size_t bytes; };
        const Opt opts[] = {{(const void*)&k_col<COL_NORMAL>, P->lds_col}, {(const void*)&k_col<COL_FWD>, P->lds_col},
                            {(const void*)&k_col<COL_ADJ>, P->lds_col}, {(const void*)&k_col<COL_REG>, P->lds_col},
                            {(const void*)&k_gram_q<16>, P->lds_gram}, {(const void*)&k_gram_q<32>, P->lds_gram},
                            {(const void*)&k_gram_q<64>, P->lds_gram}, {(const void*)&k_gram_q<128>, P->lds_gram},
                            {(const void*)&k_gram_q<256>, P->lds_gram}, {(const void*)P->band, P->lds_band},
                            {(const void*)P->band_f32, P->lds_band},
                            {(const void*)&k_gram_lines<true>, P->lds_gram_lines},
                            {(const void*)&k_gram_lines<false>, P->lds_gram_lines},
                            {(const void*)&k_gram_q_any, P->lds_gram}};
        for (const Opt& o : opts)
            if (hipFuncSetAttribute(o.f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)o.bytes) != hipSuccess)
                ok = false;
        if (P->col_fast >= 0 && (hipFuncSetAttribute(kColFast[P->col_fast].fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)P->lds_colfast) != hipSuccess ||
                                 hipFuncSetAttribute(kColFast[P->col_fast].fn_f32,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)P->lds_colfast) != hipSuccess))
            ok = false;
        if (P->col_mix >= 0 && hipFuncSetAttribute(kColMix[P->col_mix].fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)P->lds_colmix) != hipSuccess)
            ok = false;
    }
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        (void)hipFree(P->arena);
        delete P;
        return SMSM_E_DEVICE;
    }
    *out = P;
    return SMSM_OK;
}

smsm_status smsm_plan_destroy(smsm_plan* plan) {
    if (!plan) return SMSM_OK;
    (void)hipSetDevice(plan->dev);
    (void)hipDeviceSynchronize();
    for (hipEvent_t ev : plan->kt_ev) (void)hipEventDestroy(ev);
    (void)hipFree(plan->arena);
    delete plan;
    return SMSM_OK;
}

size_t smsm_plan_device_bytes(const smsm_plan* plan) { return plan ? plan->bytes : 0; }

size_t smsm_workspace_bytes(const smsm_plan* plan) { return plan ? plan->ws_bytes : 0; }

smsm_status smsm_set_workspace(smsm_plan* plan, void* ws_dev, size_t bytes) {
    if (!plan) return SMSM_E_INVALID;
    if (ws_dev && (bytes < plan->ws_bytes || (reinterpret_cast<uintptr_t>(ws_dev) & 255u) != 0))
        return SMSM_E_INVALID;
    bind_workspace(plan, ws_dev);
    return SMSM_OK;
}

smsm_status smsm_plan_set_params(smsm_plan* plan, const smsm_params* params) {
    if (!plan) return SMSM_E_INVALID;
    smsm_status s = check_params(params);
    if (s) return s;
    const int nit = params->ns_max_iter > 0 ? params->ns_max_iter : kNsDefaultIters;
    if (nit > plan->ns_iters) return SMSM_E_UNSUPPORTED;   // done-flag array sized at creation
    if ((params->flags & SMSM_FLAG_GRAM_BF16) && !plan->gram_bf16_ws) return SMSM_E_UNSUPPORTED;
    plan->prm = *params;
    plan->ns_iters = nit;
    return SMSM_OK;
}

smsm_status smsm_solve(smsm_plan* P, const void* y_dev, void* x_dev, void* stream) {
    if (!P || !y_dev || !x_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    const Geo& g = P->g;
    const size_t nvec = (size_t)g.L * g.Ns * g.n2 * g.n1;
    const size_t ny = (size_t)g.Ns * g.Nc * g.n2 * g.n1 * sizeof(float2);
    const bool c128 = (P->prm.flags & SMSM_FLAG_X_C128) != 0;
    const size_t nx = nvec * (c128 ? sizeof(double2) : sizeof(float2));
    if (overlap(y_dev, ny, x_dev, nx)) return SMSM_E_INVALID;
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    hipStream_t st = S(stream);
    const smsm_params& prm = P->prm;
    const bool reg = prm.lambda > 0.0;
    smsm_status s;

    // CG runs on the hybrid layout (x image, ky k-space); the kx transform is
    // unitary, so iterates, inner products and step lengths are those of the
    // natural-domain CG.
    const long nvec_l = (long)nvec;
    if ((s = chain_AH_hyb(P, (const float2*)y_dev, P->b, st))) return s;
    hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, nvec_l, P->b, P->x);
    LAUNCH_CHECK();
    double* RR[3] = {P->pr, P->pr + P->npr, P->pr + 2 * P->npr};   // |r|^2 partials of the last three residuals
    for (int k = 0; k < prm.n_irls; ++k) {
        if (reg) {
            // Gram of the natural iterate (the hybrid one feeds its column pass)
            if ((s = rows_fwd(P, P->x, P->q, st))) return s;
            if ((s = chain_gram(P, P->q, P->x, P->G, st))) return s;
            if (k == 0 && (s = chain_lmax(P, P->G, P->sigma, st))) return s;
            const double frac = std::max(prm.eps_frac * std::pow(prm.eps_decay, -(double)k), prm.eps_floor_frac);
            if ((s = chain_weights(P, P->G, P->sigma, frac, st))) return s;
            if ((s = band_tables(P, st))) return s;
        }
        HybArgs a0{};
        a0.mode = 1;
        a0.bvec = P->b;
        a0.out = P->r;
        a0.part = RR[0];
        if ((s = hyb_apply(P, P->x, COL_NORMAL, reg, a0, st))) return s;
        for (int j = 0; j < prm.n_cg; ++j) {
            // x takes step j - 1 in the column pass of step j (which reads that
            // direction anyway) and the last step after the loop
            ColCg pc{};
            pc.r = P->r;
            pc.p_old = P->p;
            pc.p = P->p;
            pc.x = P->x;
            pc.alpha_prev = P->cgs + 8;
            pc.rr_new = RR[j % 3];
            pc.nrr = P->npr;
            pc.rr_old = P->cgs + (j + 2) % 3;
            pc.rr_out = P->cgs + j % 3;
            pc.mode = j == 0 ? 1 : 2;
            pc.pq = P->pq;
            if ((s = col<COL_NORMAL>(P, nullptr, P->h2, reg ? 1 : 0, pc, st))) return s;
            if (reg) {
                if ((s = band_extract(P, P->p, P->col_fast < 0, st))) return s;
                if ((s = band_corr(P, st))) return s;
            }
            HybArgs a{};
            a.mode = 2;
            a.rr = P->cgs + j % 3;
            a.use_band = reg ? 1 : 0;
            a.h2 = P->h2;
            a.r = P->r;
            a.part = RR[(j + 1) % 3];
            if ((s = hyb_update(P, a, st))) return s;
        }
        if (prm.n_cg > 0 && (s = x_step(P, st))) return s;
    }
    if ((s = rows_fwd(P, P->x, P->q, st))) return s;
    if (c128)
        hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, nvec_l, P->q, (double2*)x_dev);
    else
        hipLaunchKernelGGL(k_to_c64, vec_grid(), dim3(kThreads), 0, st, nvec_l, P->q, (float2*)x_dev);
    LAUNCH_CHECK();
    return SMSM_OK;
}

}  // extern "C"

// ---- the solve without allocation: a static device array as the workspace --
// One array per device (each device that loads the library holds its own copy
// until the process ends).  Host code must not pass `scratch` itself to a
// kernel: its device address comes from hipGetSymbolAddress, taken once per
// device with that device current and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[SMSM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of this device's scratch (the current device must be `dev`).
smsm_status scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kScratchDevices) return SMSM_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SMSM_E_DEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SMSM_OK;
}
}  // namespace

extern "C" {

smsm_status smsm_solve_noalloc(smsm_plan* P, const void* y_dev, void* x_dev, void* stream) {
    if (!P || !y_dev || !x_dev) return SMSM_E_INVALID;
    if (P->ws_bytes > (size_t)SMSM_NOALLOC_SCRATCH_BYTES) return SMSM_E_SCRATCH;
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    void* base = nullptr;
    smsm_status s = scratch_address(P->dev, &base);
    if (s) return s;
    // the solve runs in the scratch (every buffer it reads it writes first, so
    // nothing needs clearing); the plan's own binding comes back afterwards
    void* own = P->ws;
    const bool own_weights = P->have_weights;
    bind_workspace(P, base);
    s = smsm_solve(P, y_dev, x_dev, stream);
    bind_workspace(P, own);
    P->have_weights = own_weights;
    return s;
}

smsm_status smsm_plan_status(smsm_plan* P) {
    if (!P) return SMSM_E_INVALID;
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return SMSM_E_DEVICE;
    int h[2] = {0, 0};
    if (hipMemcpy(h, P->flags, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return SMSM_E_DEVICE;
    const int zero[2] = {0, 0};
    if (hipMemcpy(P->flags, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) return SMSM_E_DEVICE;
    return h[0] ? SMSM_E_NUMERIC : (h[1] ? SMSM_E_NOT_CONVERGED : SMSM_OK);
}

smsm_status smsm_apply_A(smsm_plan* P, const void* x_dev, void* y_dev, void* stream) {
    if (!P || !x_dev || !y_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    const Geo& g = P->g;
    hipStream_t st = S(stream);
    const long ny = (long)g.Ns * g.Nc * g.n2 * g.n1;
    hipLaunchKernelGGL(k_zero_c128, vec_grid(), dim3(kThreads), 0, st, ny, (double2*)y_dev);
    LAUNCH_CHECK();
    smsm_status s = rows_inv(P, (const double2*)x_dev, P->h1, st);
    if (s) return s;
    if ((s = col<COL_FWD>(P, P->h1, P->h2, 0, no_cg(), st))) return s;
    hipLaunchKernelGGL(k_yrows_fwd, dim3(g.M / P->TRy, g.Ns * g.Nc), dim3(kThreads), P->lds_rows, st, g,
                       P->ytil, (double2*)y_dev, P->tw1, P->TRy);
    LAUNCH_CHECK();
    return SMSM_OK;
}

smsm_status smsm_apply_AH(smsm_plan* P, const void* y_dev, void* x_dev, void* stream) {
    if (!P || !y_dev || !x_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    hipStream_t st = S(stream);
    smsm_status s = chain_AH_hyb(P, (const float2*)y_dev, P->h2, st);
    if (s) return s;
    return rows_fwd(P, P->h2, (double2*)x_dev, st);
}

smsm_status smsm_apply_AHA(smsm_plan* P, const void* x_dev, void* out_dev, void* stream) {
    if (!P || !x_dev || !out_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    return chain_normal(P, (const double2*)x_dev, (double2*)out_dev, COL_NORMAL, false, S(stream));
}

smsm_status smsm_gram(smsm_plan* P, const void* x_dev, void* g_dev, void* stream) {
    if (!P || !x_dev || !g_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    return chain_gram(P, (const double2*)x_dev, nullptr, (double2*)g_dev, S(stream));
}

smsm_status smsm_weights(smsm_plan* P, const void* g_dev, const double* eps, void* w_dev, void* stream) {
    if (!P || !g_dev || !eps || !w_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    const Geo& g = P->g;
    hipStream_t st = S(stream);
    if (hipMemcpyAsync(P->epsin, eps, g.L * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
        return SMSM_E_DEVICE;
    smsm_status s = chain_weights(P, (const double2*)g_dev, P->epsin, 1.0, st);
    if (s) return s;
    if (hipMemcpyAsync(w_dev, P->W, (size_t)g.L * g.K * g.K * sizeof(double2), hipMemcpyDeviceToDevice, st) !=
        hipSuccess)
        return SMSM_E_DEVICE;
    return hipStreamSynchronize(st) == hipSuccess ? SMSM_OK : SMSM_E_DEVICE;
}

smsm_status smsm_lambda_max(smsm_plan* P, const void* g_dev, void* lmax_dev, void* stream) {
    if (!P || !g_dev || !lmax_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    return chain_lmax(P, (const double2*)g_dev, (double*)lmax_dev, S(stream));
}

smsm_status smsm_set_weights(smsm_plan* P, const void* w_dev, void* stream) {
    if (!P || !w_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    const Geo& g = P->g;
    hipStream_t st = S(stream);
    if (hipMemcpyAsync(P->W, w_dev, (size_t)g.L * g.K * g.K * sizeof(double2), hipMemcpyDeviceToDevice, st) !=
        hipSuccess)
        return SMSM_E_DEVICE;
    return band_tables(P, st);
}

smsm_status smsm_apply_reg(smsm_plan* P, const void* x_dev, void* out_dev, void* stream) {
    if (!P || !x_dev || !out_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (!P->have_weights) return SMSM_E_INVALID;
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    return chain_normal(P, (const double2*)x_dev, (double2*)out_dev, COL_REG, true, S(stream));
}

smsm_status smsm_apply_normal(smsm_plan* P, const void* x_dev, void* out_dev, void* stream) {
    if (!P || !x_dev || !out_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (!P->have_weights) return SMSM_E_INVALID;
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    return chain_normal(P, (const double2*)x_dev, (double2*)out_dev, COL_NORMAL, true, S(stream));
}

// ---- batches of solves under one graph -----------------------------------
struct smsm_batch {
    int dev = 0;
    int n_streams = 0;
    std::vector<hipGraph_t> graphs;         // consecutive segments of the entries, launched in order
    std::vector<hipGraphExec_t> execs;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
};

static void batch_release(smsm_batch* B) {
    for (hipGraphExec_t e : B->execs) (void)hipGraphExecDestroy(e);
    for (hipGraph_t gr : B->graphs) (void)hipGraphDestroy(gr);
    for (hipEvent_t ev : B->events) (void)hipEventDestroy(ev);
    for (hipStream_t st : B->streams) (void)hipStreamDestroy(st);
    delete B;
}

static smsm_status batch_capture(smsm_plan* const* plans, int n, const void* const* y_devs, void* const* x_devs,
                                 int n_streams, smsm_batch** out);

// Times one launch of a captured batch (after one untimed launch), in ms.
static smsm_status batch_time(smsm_batch* B, hipStream_t st, float* ms) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SMSM_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return SMSM_E_DEVICE; }
    auto launch_all = [&]() {
        for (hipGraphExec_t e : B->execs)
            if (hipGraphLaunch(e, st) != hipSuccess) return false;
        return true;
    };
    bool ok = launch_all() && hipEventRecord(e0, st) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k) ok = launch_all();
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(ms, e0, e1) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ok ? SMSM_OK : SMSM_E_DEVICE;
}

smsm_status smsm_batch_create(smsm_plan* const* plans, int n, const void* const* y_devs, void* const* x_devs,
                              int n_streams, smsm_batch** out) {
    if (!out || n_streams < 0 || n_streams > 64) return SMSM_E_INVALID;
    if (n_streams > 0) return batch_capture(plans, n, y_devs, x_devs, n_streams, out);
    // autotune the stream count: capture each candidate, time it, keep the fastest
    *out = nullptr;
    static const int kCand[] = {1, 2, 3, 4, 6, 8};
    smsm_batch* best = nullptr;
    float best_ms = 0.0f;
    hipStream_t st = nullptr;
    int distinct = 0;
    for (int k = 0; k < n; ++k) {
        bool seen = false;
        for (int j = 0; j < k && !seen; ++j) seen = plans && plans[j] == plans[k];
        distinct += seen ? 0 : 1;
    }
    for (int c : kCand) {
        if (c > distinct && c != 1) break;
        smsm_batch* B = nullptr;
        smsm_status s = batch_capture(plans, n, y_devs, x_devs, c, &B);
        if (s == SMSM_OK && !st && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            st = nullptr;
            s = SMSM_E_DEVICE;
        }
        float ms = 0.0f;
        if (s == SMSM_OK) s = batch_time(B, st, &ms);
        if (s != SMSM_OK) {
            if (B) batch_release(B);
            if (best) batch_release(best);
            if (st) (void)hipStreamDestroy(st);
            return s;
        }
        if (!best || ms < best_ms) {
            if (best) batch_release(best);
            best = B;
            best_ms = ms;
        } else {
            batch_release(B);
        }
    }
    if (st) (void)hipStreamDestroy(st);
    *out = best;
    return SMSM_OK;
}

int smsm_batch_streams(const smsm_batch* batch) { return batch ? batch->n_streams : 0; }

static smsm_status batch_capture(smsm_plan* const* plans, int n, const void* const* y_devs, void* const* x_devs,
                                 int n_streams, smsm_batch** out) {
    if (!plans || !y_devs || !x_devs || !out || n < 1 || n_streams < 1 || n_streams > 64) return SMSM_E_INVALID;
    *out = nullptr;
    // a plan's solves share its scratch memory: they all go, in order, to the
    // stream of its first entry; distinct plans are dealt round-robin
    std::vector<int> owner(n);
    int distinct = 0;
    for (int k = 0; k < n; ++k) {
        if (!plans[k] || !y_devs[k] || !x_devs[k]) return SMSM_E_INVALID;
        if (!plans[k]->ws) return SMSM_E_INVALID;            // the graph bakes in the bound workspace
        if (plans[k]->dev != plans[0]->dev) return SMSM_E_INVALID;
        if (plans[k]->kt_cap > 0) return SMSM_E_INVALID;      // no per-launch timing inside a graph
        owner[k] = -1;
        for (int j = 0; j < k && owner[k] < 0; ++j)
            if (plans[j] == plans[k]) owner[k] = owner[j];
        if (owner[k] < 0) owner[k] = distinct++;
    }
    if (hipSetDevice(plans[0]->dev) != hipSuccess) return SMSM_E_DEVICE;
    smsm_batch* B = new (std::nothrow) smsm_batch;
    if (!B) return SMSM_E_NOMEM;
    B->dev = plans[0]->dev;
    const int ns = std::min(n_streams, distinct);
    B->n_streams = ns;
    for (int k = 0; k < ns; ++k) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) { batch_release(B); return SMSM_E_DEVICE; }
        B->streams.push_back(st);
    }
    for (int k = 0; k < ns; ++k) {   // event 0 forks, events 1.. join
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) { batch_release(B); return SMSM_E_DEVICE; }
        B->events.push_back(ev);
    }
    // consecutive segments of at most kBatchMaxSegment entries in which no
    // plan has more than kBatchMaxRepeat, each captured as its own graph (fork from and join into the
    // first stream) and launched in order: a plan's solves run in sequence on
    // one stream, so a segment bounds the length of the graph's dependency
    // chains
    hipStream_t origin = B->streams[0];
    std::vector<int> count(distinct, 0);
    int k0 = 0;
    while (k0 < n) {
        std::fill(count.begin(), count.end(), 0);
        int k1 = k0;
        while (k1 < n && k1 - k0 < kBatchMaxSegment && count[owner[k1]] < kBatchMaxRepeat) ++count[owner[k1++]];
        if (hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            batch_release(B);
            return SMSM_E_DEVICE;
        }
        bool ok = hipEventRecord(B->events[0], origin) == hipSuccess;
        for (int k = 1; k < ns && ok; ++k) ok = hipStreamWaitEvent(B->streams[k], B->events[0], 0) == hipSuccess;
        smsm_status s = ok ? SMSM_OK : SMSM_E_DEVICE;
        for (int k = k0; k < k1 && s == SMSM_OK; ++k)
            s = smsm_solve(plans[k], y_devs[k], x_devs[k], B->streams[owner[k] % ns]);
        for (int k = 1; k < ns && s == SMSM_OK; ++k) {
            if (hipEventRecord(B->events[k], B->streams[k]) != hipSuccess ||
                hipStreamWaitEvent(origin, B->events[k], 0) != hipSuccess)
                s = SMSM_E_DEVICE;
        }
        hipGraph_t graph = nullptr;
        const bool ended = hipStreamEndCapture(origin, &graph) == hipSuccess;
        if (graph) B->graphs.push_back(graph);
        if (s != SMSM_OK || !ended || !graph) {
            batch_release(B);
            return s != SMSM_OK ? s : SMSM_E_DEVICE;
        }
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            batch_release(B);
            return SMSM_E_DEVICE;
        }
        B->execs.push_back(exec);
        k0 = k1;
    }
    *out = B;
    return SMSM_OK;
}

smsm_status smsm_batch_launch(smsm_batch* B, void* stream) {
    if (!B) return SMSM_E_INVALID;
    if (hipSetDevice(B->dev) != hipSuccess) return SMSM_E_DEVICE;
    for (hipGraphExec_t e : B->execs)
        if (hipGraphLaunch(e, S(stream)) != hipSuccess) return SMSM_E_DEVICE;
    return SMSM_OK;
}

smsm_status smsm_batch_destroy(smsm_batch* B) {
    if (!B) return SMSM_OK;
    (void)hipSetDevice(B->dev);
    (void)hipDeviceSynchronize();
    batch_release(B);
    return SMSM_OK;
}

smsm_status smsm_plan_autotune(smsm_plan* P, int reps, int* shape, void* stream) {
    if (!P || reps < 1 || reps > 1000) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    hipStream_t st = S(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SMSM_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SMSM_E_DEVICE;
    }
    // ms for `reps` rounds of the kernels of `ids`, after one untimed round
    auto timed = [&](const int* ids, int nid, float* ms) -> smsm_status {
        for (int round = 0; round < 2; ++round) {
            if (round == 1 && hipEventRecord(e0, st) != hipSuccess) return SMSM_E_DEVICE;
            for (int k = 0; k < nid; ++k) {
                smsm_status s = smsm_launch_kernel(P, ids[k], round == 0 ? 1 : reps, stream);
                if (s) return s;
            }
        }
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return SMSM_E_DEVICE;
        return SMSM_OK;
    };
    smsm_status s = SMSM_OK;
    static const int kTrw[] = {2, 4, 8, 16, 32};
    static const int kXw[] = {1, 2, 4};
    const int rows_ids[] = {SMSM_KERNEL_ROWS_INV, SMSM_KERNEL_ROWS_FWD};
    const int vec_ids[] = {SMSM_KERNEL_CG_UPDATE};
    int best_trw = P->TRw, best_xw = P->hyb_xw;
    float best = 0.0f;
    bool any = false;
    for (int trw : kTrw) {
        if (s || !is_pow2(P->g.n1) || !rows_shape_ok(P->g, trw)) continue;
        set_rows_shape(P, trw);
        float ms = 0.0f;
        s = timed(rows_ids, 2, &ms);
        if (!s && (!any || ms < best)) {
            best = ms;
            best_trw = trw;
            any = true;
        }
    }
    set_rows_shape(P, best_trw);
    any = false;
    for (int xw : kXw) {
        if (s || !set_hyb_shape(P, xw)) continue;
        float ms = 0.0f;
        s = timed(vec_ids, 1, &ms);
        if (!s && (!any || ms < best)) {
            best = ms;
            best_xw = xw;
            any = true;
        }
    }
    (void)set_hyb_shape(P, best_xw);
    // the timed launches ran on whatever the buffers held: forget what they flagged
    if (!s && (hipMemsetAsync(P->flags, 0, 4 * sizeof(int), st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess))
        s = SMSM_E_DEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!s && shape) {
        shape[0] = P->TRw;
        shape[1] = P->hyb_xw;
    }
    return s;
}

smsm_status smsm_kernel_timer_start(smsm_plan* P, int kernel_id, int capacity, int stride) {
    if (!P || capacity < 0 || capacity > (1 << 20) || stride < 1) return SMSM_E_INVALID;
    if (kernel_id != SMSM_KERNEL_COL_NORMAL) return SMSM_E_UNSUPPORTED;
    if (capacity > 0 && P->col_fast < 0) return SMSM_E_UNSUPPORTED;
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    P->kt_cap = P->kt_n = P->kt_seen = 0;
    P->kt_stride = stride;
    const size_t need = 2 * (size_t)capacity;
    while (P->kt_ev.size() > need) {
        (void)hipEventDestroy(P->kt_ev.back());
        P->kt_ev.pop_back();
    }
    while (P->kt_ev.size() < need) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return SMSM_E_DEVICE;
        P->kt_ev.push_back(ev);
    }
    P->kt_cap = capacity;
    return SMSM_OK;
}

smsm_status smsm_kernel_timer_read(smsm_plan* P, double* total_ms, int* launches) {
    if (!P || !total_ms || !launches) return SMSM_E_INVALID;
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    double tot = 0.0;
    const int n = P->kt_n;
    if (n > 0 && hipEventSynchronize(P->kt_ev[2 * (n - 1) + 1]) != hipSuccess) return SMSM_E_DEVICE;
    for (int k = 0; k < n; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, P->kt_ev[2 * k], P->kt_ev[2 * k + 1]) != hipSuccess) return SMSM_E_DEVICE;
        tot += ms;
    }
    *total_ms = tot;
    *launches = n;
    P->kt_n = 0;
    return SMSM_OK;
}

smsm_status smsm_images_sos(smsm_plan* P, const void* x_dev, void* img_dev, void* stream) {
    if (!P || !x_dev || !img_dev) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    const Geo& g = P->g;
    hipStream_t st = S(stream);
    smsm_status s = rows_inv(P, (const double2*)x_dev, P->h1, st);
    if (s) return s;
    const dim3 grid(g.n1, g.L);
    double* img = (double*)img_dev;
    if (!is_pow2(g.n2)) {
        hipLaunchKernelGGL(k_sos_any, grid, dim3(kThreads), (size_t)(g.Ns + 1) * g.n2 * sizeof(double2), st, g,
                           P->h1, P->tw2, img);
    } else switch (g.n2) {
        case 16: hipLaunchKernelGGL(k_sos_cols<16>, grid, dim3(64), 0, st, g, P->h1, P->tw2, img); break;
        case 32: hipLaunchKernelGGL(k_sos_cols<32>, grid, dim3(64), 0, st, g, P->h1, P->tw2, img); break;
        case 64: hipLaunchKernelGGL(k_sos_cols<64>, grid, dim3(64), 0, st, g, P->h1, P->tw2, img); break;
        case 128: hipLaunchKernelGGL(k_sos_cols<128>, grid, dim3(64), 0, st, g, P->h1, P->tw2, img); break;
        default: hipLaunchKernelGGL(k_sos_cols<256>, grid, dim3(64), 0, st, g, P->h1, P->tw2, img); break;
    }
    LAUNCH_CHECK();
    return SMSM_OK;
}

}  // extern "C"

namespace {

// Algorithmic FP64 flops and compulsory bytes of one launch (see smsm.h).
void kernel_cost(const Geo& g, int id, bool khat_f32, double* flops, double* bytes) {
    const double n1 = g.n1, n2 = g.n2, B = g.B, L = g.L, Ns = g.Ns, Nc = g.Nc, M = g.M, nc = g.nc, e = g.e;
    const double vec = B * n1 * n2 * 16.0;               // one c128 vector
    const double ds = band_ds(g.Ns, g.nc);
    auto F = [](double n) { return 5.0 * n * std::log2(n); };
    double f = 0.0, b = 0.0;
    switch (id) {
        case SMSM_KERNEL_COL_NORMAL: {
            const double per_col =
                2.0 * B * F(n2)                                   // ky inverse + forward DFT
                + 6.0 * B * n2 * 2.0                              // tau modulation and final scaling
                + Nc * (8.0 * B * n2                              // fold
                        + 2.0 * B * F(M)                          // pruned DFT + inverse
                        + Ns * M * L * 14.0                       // CAIPI slice sum and split
                        + 8.0 * B * n2)                           // unfold-accumulate
                + B * n2 * Ns * 8.0                               // per-pixel Hankel term (Ns taps)
                + B * n2 * 12.0;                                  // x += alpha p, p = r + beta p, Re <p, q>
            f = n1 * per_col;
            b = 6.0 * vec + L * Nc * n1 * n2 * 16.0                // r, p, x in; p, q, x out; coil maps (c128)
                + L * Ns * (Ns + 1) / 2.0 * n1 * n2 * (khat_f32 ? 8.0 : 16.0);   // image-domain Hankel kernel (pairs j <= i)
            break;
        }
        case SMSM_KERNEL_ROWS_INV:
        case SMSM_KERNEL_ROWS_FWD:
            f = B * n2 * F(n1);
            b = 2.0 * vec;
            break;
        case SMSM_KERNEL_BAND_CORR: {
            f = 8.0 * B * (2.0 * e * n2 * nc * nc + 2.0 * e * n1 * nc + 4.0 * e * e * nc * nc) * Ns;
            b = L * 2.0 * e * Ns * Ns * nc * nc * 16.0                     // column-side tables
                + L * 4.0 * e * e * Ns * Ns * nc * nc * (khat_f32 ? 8.0 : 16.0)   // corner tables
                + L * 2.0 * e * Ns * nc * Ns * n1 * (khat_f32 ? 8.0 : 16.0)      // transformed row tables
                + B * 4.0 * e * n2 * 16.0 + B * 2.0 * e * nc * n1 * 16.0    // band columns, rows of p
                + B * (ds * 2.0 * e * n2 + 2.0 * e * n1 + 4.0 * e * e) * 16.0;   // corrections out
            break;
        }
        case SMSM_KERNEL_CG_UPDATE:
            f = B * n1 * n2 * (10.0 + 8.0 * 2.0 * e);
            b = 3.0 * vec + B * (ds * 2.0 * e * n2 + 2.0 * e * n1 + 4.0 * e * e) * 16.0;
            break;
        case SMSM_KERNEL_BAND_EXTRACT:
            f = 8.0 * B * n1 * n2 * 4.0 * e;
            b = vec + B * 4.0 * e * n2 * 16.0;
            break;
        default:
            break;
    }
    (void)nc;
    *flops = f;
    *bytes = b;
}

}  // namespace

extern "C" {

smsm_status smsm_kernel_cost(const smsm_plan* P, int id, double* flops, double* bytes) {
    if (!P || !flops || !bytes || id < 0 || id > SMSM_KERNEL_BAND_EXTRACT) return SMSM_E_INVALID;
    kernel_cost(P->g, id, P->khat_f32, flops, bytes);
    return SMSM_OK;
}

smsm_status smsm_launch_kernel(smsm_plan* P, int id, int reps, void* stream) {
    if (!P || reps < 0 || id < 0 || id > SMSM_KERNEL_BAND_EXTRACT) return SMSM_E_INVALID;
    if (!P->ws) return SMSM_E_INVALID;   // no workspace bound
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    hipStream_t st = S(stream);
    const bool reg = P->prm.lambda > 0.0 && P->have_weights;
    for (int k = 0; k < reps; ++k) {
        smsm_status s = SMSM_OK;
        switch (id) {
            case SMSM_KERNEL_COL_NORMAL: {
                ColCg pc{};
                pc.r = P->r;
                pc.p_old = P->p;
                pc.p = P->p;
                pc.x = P->x;
                pc.alpha_prev = P->cgs + 8;
                pc.rr_new = P->pr + P->npr;
                pc.nrr = P->npr;
                pc.rr_old = P->cgs;
                pc.rr_out = P->cgs + 1;
                pc.mode = 2;
                pc.pq = P->pq;
                s = col<COL_NORMAL>(P, nullptr, P->h2, reg ? 1 : 0, pc, st);
                break;
            }
            case SMSM_KERNEL_ROWS_INV: s = rows_inv(P, P->q, P->h1, st); break;
            case SMSM_KERNEL_ROWS_FWD: s = rows_fwd(P, P->x, P->q, st); break;
            case SMSM_KERNEL_BAND_CORR: s = band_corr(P, st); break;
            case SMSM_KERNEL_BAND_EXTRACT: s = band_extract(P, P->p, P->col_fast < 0, st); break;
            case SMSM_KERNEL_CG_UPDATE: {
                HybArgs a{};
                a.mode = 2;
                a.rr = P->cgs + 1;
                a.use_band = reg ? 1 : 0;
                a.h2 = P->h2;
                a.r = P->r;
                a.part = P->pr + 2 * P->npr;
                s = hyb_update(P, a, st);
                break;
            }
        }
        if (s) return s;
    }
    return SMSM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned unrolled solver (network and workspace for one plan's geometry).
// ---------------------------------------------------------------------------

struct smsm_learned {
    smsm_plan* P = nullptr;
    int dev = 0;
    int width = 0, nc = 0, L = 0, H = 0, W = 0;   // nc = 2 Ns channels in and out
    int n_unroll = 0, n_cg = 0;
    double mu = 0.0;
    static constexpr int kDepth = 5;
    int cin[kDepth] = {}, cout[kDepth] = {};
    size_t woff[kDepth] = {}, boff[kDepth] = {};
    size_t nparam = 0;
    long adam_t = 0;
    void* arena = nullptr;
    float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
    float* act[kDepth + 1] = {};          // act[0] network input, act[k] output of layer k-1, act[5] output
    float *ga = nullptr, *gbuf = nullptr, *gio = nullptr;   // hidden-gradient ping-pong, nc-channel gradient
    double2 *b = nullptr, *x = nullptr, *z = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *rhs = nullptr;
    double2 *g = nullptr, *wv = nullptr, *ax = nullptr, *xs = nullptr;
    double *part = nullptr, *scal = nullptr;   // scal: [0] s, [1] and [4] rr, [2] alpha, [3] beta, [8] loss num, [9] den
    double* part2 = nullptr;                    // second partials buffer of the fused CG steps
    float *wpart = nullptr, *wbpart = nullptr;  // weight-gradient chunk partials (k_wgrad_part)
    // 0: FP32 weights on the vector ALU; BF16 weights on the matrix cores with
    // 1: exact products (FP32 activations in three BF16 parts), 2: the BF16
    // network (convolution inputs and hidden activations rounded to BF16)
    int bf16 = 0;
    // packed BF16 weights per layer, [0] forward P[o][t][c], [1] backward-data
    // P[c][t][o] (taps flipped), refreshed after every change of the parameters
    unsigned short* wpk[kDepth][2] = {};
    int pk_rows[kDepth][2] = {}, pk_cols[kDepth][2] = {};
};

namespace {

long lvec(const smsm_learned* Lr) { return (long)Lr->L * (Lr->nc / 2) * Lr->H * Lr->W; }

template <int COB>
void lconv_k(smsm_learned* Lr, dim3 grid, int ci, int co, const float* in, const float* w, const float* bias,
             float* out, int relu, bool bwd, hipStream_t st) {
    if (bwd) hipLaunchKernelGGL((k_conv3x3<COB, 1>), grid, dim3(CNN_THREADS), 0, st, ci, co, Lr->H, Lr->W, in, w, bias, out, relu);
    else hipLaunchKernelGGL((k_conv3x3<COB, 0>), grid, dim3(CNN_THREADS), 0, st, ci, co, Lr->H, Lr->W, in, w, bias, out, relu);
}
// Layer k's convolution (bwd: its backward-data transpose, no bias): FP32
// weights on the vector ALU, or BF16 weights on the matrix cores.
smsm_status lconv(smsm_learned* Lr, int k, bool bwd, const float* in, float* out, int relu, hipStream_t st) {
    const int ci = bwd ? Lr->cout[k] : Lr->cin[k], co = bwd ? Lr->cin[k] : Lr->cout[k];
    const float* bias = bwd ? nullptr : Lr->params + Lr->boff[k];
    if (Lr->bf16) {
        const int d = bwd ? 1 : 0, rows = Lr->pk_rows[k][d];
        const dim3 grid(((Lr->H + CM_TR - 1) / CM_TR) * ((Lr->W + CM_TC - 1) / CM_TC), 1, Lr->L);
        const int cols = Lr->pk_cols[k][d], rnd = (Lr->bf16 == 2 && relu) ? 1 : 0;
        const unsigned short* P = Lr->wpk[k][d];
        const int H = Lr->H, W = Lr->W;
        if (Lr->bf16 == 2) {
            if (rows % 64 == 0)
                hipLaunchKernelGGL((k_conv3x3_mfma<4, 1>), dim3(grid.x, rows / 64, grid.z), dim3(256), 0, st, ci, co,
                                   cols, H, W, in, P, bias, out, relu, rnd);
            else
                hipLaunchKernelGGL((k_conv3x3_mfma<1, 1>), dim3(grid.x, rows / 16, grid.z), dim3(256), 0, st, ci, co,
                                   cols, H, W, in, P, bias, out, relu, rnd);
        } else {
            if (rows % 64 == 0)
                hipLaunchKernelGGL((k_conv3x3_mfma<4, 3>), dim3(grid.x, rows / 64, grid.z), dim3(256), 0, st, ci, co,
                                   cols, H, W, in, P, bias, out, relu, 0);
            else
                hipLaunchKernelGGL((k_conv3x3_mfma<1, 3>), dim3(grid.x, rows / 16, grid.z), dim3(256), 0, st, ci, co,
                                   cols, H, W, in, P, bias, out, relu, 0);
        }
        LAUNCH_CHECK();
        return SMSM_OK;
    }
    const int npx = Lr->H * Lr->W;
    const dim3 grid((npx + CNN_THREADS - 1) / CNN_THREADS, co % 8 == 0 ? co / 8 : co / 4, Lr->L);
    const float* w = Lr->params + Lr->woff[k];
    if (co % 8 == 0) lconv_k<8>(Lr, grid, ci, co, in, w, bias, out, relu, bwd, st);
    else lconv_k<4>(Lr, grid, ci, co, in, w, bias, out, relu, bwd, st);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// Refresh the packed BF16 weights of every layer (when the network uses them).
smsm_status lrefresh_bf16(smsm_learned* Lr, hipStream_t st) {
    if (!Lr->bf16) return SMSM_OK;
    for (int k = 0; k < smsm_learned::kDepth; ++k)
        for (int d = 0; d < 2; ++d) {
            hipLaunchKernelGGL(k_conv_wpack, dim3(256), dim3(kThreads), 0, st, Lr->cin[k], Lr->cout[k],
                               Lr->params + Lr->woff[k], d, Lr->pk_rows[k][d], Lr->pk_cols[k][d], Lr->wpk[k][d]);
            LAUNCH_CHECK();
        }
    return SMSM_OK;
}

// act[0] -> act[1..5] (ReLU after layers 0..3).  The BF16 network first
// rounds its input act[0] to BF16 values (in place).
smsm_status lcnn_forward(smsm_learned* Lr, hipStream_t st) {
    if (Lr->bf16 == 2) {
        hipLaunchKernelGGL(k_round_bf16, vec_grid(), dim3(kThreads), 0, st, (long)Lr->L * Lr->nc * Lr->H * Lr->W,
                           Lr->act[0]);
        LAUNCH_CHECK();
    }
    for (int k = 0; k < smsm_learned::kDepth; ++k) {
        smsm_status s = lconv(Lr, k, false, Lr->act[k], Lr->act[k + 1], k < smsm_learned::kDepth - 1, st);
        if (s) return s;
    }
    return SMSM_OK;
}

// Given the activations of a forward pass and the gradient gout of the
// output (nc channels), the weight gradients (accumulated when asked) and
// the gradient of the input in gin (nc channels).
smsm_status lcnn_backward(smsm_learned* Lr, const float* gout, float* gin, int accumulate, hipStream_t st) {
    const int D = smsm_learned::kDepth;
    const long nh = (long)Lr->L * Lr->width * Lr->H * Lr->W;
    const float* g = gout;
    float* bufs[2] = {Lr->ga, Lr->gbuf};
    for (int k = D - 1; k >= 0; --k) {
        if (Lr->bf16 == 2) {
            // the BF16 network: layer inputs are BF16 values, weight gradients on the matrix cores
            const int nchunk = Lr->L * wgm_chunks(Lr->H, Lr->W);
            hipLaunchKernelGGL(k_wgrad_mfma, dim3(nchunk, (Lr->cin[k] + 15) / 16), dim3(kThreads), 0, st,
                               Lr->cin[k], Lr->cout[k], Lr->H, Lr->W, Lr->act[k], g, Lr->wpart, Lr->wbpart);
            LAUNCH_CHECK();
            const int nout = Lr->cout[k] * Lr->cin[k] * 9 + Lr->cout[k];
            hipLaunchKernelGGL(k_wgrad_sum, dim3((nout + WGS_OUT - 1) / WGS_OUT), dim3(WGS_OUT, WGS_SLICES), 0, st,
                               nchunk, Lr->cin[k], Lr->cout[k], Lr->wpart, Lr->wbpart, Lr->grads + Lr->woff[k],
                               Lr->grads + Lr->boff[k], accumulate);
        } else if (Lr->cin[k] % WG_TILE == 0 && Lr->cout[k] % WG_TILE == 0) {
            const int nchunk = Lr->L * wg_chunks(Lr->H, Lr->W);
            hipLaunchKernelGGL(k_wgrad_part, dim3(nchunk, Lr->cout[k] / WG_TILE, Lr->cin[k] / WG_TILE),
                               dim3(CNN_THREADS), 0, st, Lr->cin[k], Lr->cout[k], Lr->H, Lr->W, Lr->act[k], g,
                               Lr->wpart, Lr->wbpart);
            LAUNCH_CHECK();
            const int nout = Lr->cout[k] * Lr->cin[k] * 9 + Lr->cout[k];
            hipLaunchKernelGGL(k_wgrad_sum, dim3((nout + WGS_OUT - 1) / WGS_OUT), dim3(WGS_OUT, WGS_SLICES), 0, st,
                               nchunk, Lr->cin[k], Lr->cout[k], Lr->wpart, Lr->wbpart, Lr->grads + Lr->woff[k],
                               Lr->grads + Lr->boff[k], accumulate);
        } else {
            hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(Lr->cin[k] * Lr->cout[k]), dim3(CNN_THREADS), 0, st, Lr->L,
                               Lr->cin[k], Lr->cout[k], Lr->H, Lr->W, Lr->act[k], g, Lr->grads + Lr->woff[k],
                               Lr->grads + Lr->boff[k], accumulate);
        }
        LAUNCH_CHECK();
        float* dst = k > 0 ? bufs[k & 1] : gin;
        smsm_status s = lconv(Lr, k, true, g, dst, 0, st);
        if (s) return s;
        if (k > 0) {
            hipLaunchKernelGGL(k_relu_bwd, vec_grid(), dim3(kThreads), 0, st, nh, dst, Lr->act[k]);
            LAUNCH_CHECK();
        }
        g = dst;
    }
    return SMSM_OK;
}

smsm_status ldot(smsm_learned* Lr, const double2* a, const double2* b, hipStream_t st) {
    hipLaunchKernelGGL(k_dc_dot, vec_grid(), dim3(kThreads), 0, st, lvec(Lr), a, b, Lr->part);
    LAUNCH_CHECK();
    return SMSM_OK;
}
smsm_status lscalar(smsm_learned* Lr, int mode, double* rr, double count, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_dc_scalar, dim3(1), dim3(kThreads), 0, st, mode, Lr->part, kVecBlocks, rr, count, out);
    LAUNCH_CHECK();
    return SMSM_OK;
}
smsm_status laxpy(smsm_learned* Lr, const double2* a, const double2* b, const double* fp, double fm, double2* out,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_dc_axpy, vec_grid(), dim3(kThreads), 0, st, lvec(Lr), a, b, fp, fm, out);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// out = (A^H A + mu I) v
smsm_status lnormal(smsm_learned* Lr, const double2* v, double2* out, hipStream_t st) {
    smsm_status s = chain_normal(Lr->P, v, out, COL_NORMAL, false, st);
    if (s) return s;
    return laxpy(Lr, out, v, nullptr, Lr->mu, out, st);
}

// n_cg CG steps on (A^H A + mu I) x = rhs from the x given; step lengths
// and |r|^2 stay on the device.  rr == 0 gives zero steps.
smsm_status ldc_cg(smsm_learned* Lr, const double2* rhs, double2* x, hipStream_t st) {
    double* sc = Lr->scal;
    smsm_status s;
    if ((s = lnormal(Lr, x, Lr->q, st))) return s;
    if ((s = laxpy(Lr, rhs, Lr->q, nullptr, -1.0, Lr->r, st))) return s;          // r = rhs - M x
    hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, lvec(Lr), Lr->r, Lr->p);
    LAUNCH_CHECK();
    if ((s = ldot(Lr, Lr->r, Lr->r, st)) || (s = lscalar(Lr, 0, nullptr, 0.0, sc + 1, st))) return s;
    // each step: q = (A^H A + mu I) p with Re <p, q>; x += alpha p, r -= alpha q
    // with |r|^2; p = r + beta p.  |r|^2 alternates between scal[1] and scal[4].
    const long n = lvec(Lr);
    for (int j = 0; j < Lr->n_cg; ++j) {
        double* rr_cur = (j & 1) ? sc + 4 : sc + 1;
        double* rr_next = (j & 1) ? sc + 1 : sc + 4;
        if ((s = chain_normal(Lr->P, Lr->p, Lr->q, COL_NORMAL, false, st))) return s;
        hipLaunchKernelGGL(k_dc_qdot, vec_grid(), dim3(kThreads), 0, st, n, Lr->p, Lr->q, Lr->mu, Lr->part);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_dc_xr, vec_grid(), dim3(kThreads), 0, st, n, x, Lr->r, Lr->p, Lr->q, Lr->part,
                           kVecBlocks, rr_cur, Lr->part2);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_dc_p, vec_grid(), dim3(kThreads), 0, st, n, Lr->r, Lr->p, Lr->part2, kVecBlocks, rr_cur,
                           rr_next);
        LAUNCH_CHECK();
    }
    return SMSM_OK;
}

// b = A^H y, s = sqrt(mean |b|^2).
smsm_status lsetup(smsm_learned* Lr, const void* y_dev, hipStream_t st) {
    smsm_plan* P = Lr->P;
    smsm_status s = chain_AH_hyb(P, (const float2*)y_dev, P->h2, st);
    if (s) return s;
    if ((s = rows_fwd(P, P->h2, Lr->b, st))) return s;
    if ((s = ldot(Lr, Lr->b, Lr->b, st))) return s;
    return lscalar(Lr, 3, nullptr, (double)lvec(Lr), Lr->scal, st);
}

// The unrolled forward pass from b into x (keeping x_k in xs when keep).
smsm_status lforward(smsm_learned* Lr, bool keep, hipStream_t st) {
    const long n = lvec(Lr);
    const int ns = Lr->nc / 2, npx = Lr->H * Lr->W;
    smsm_status s;
    hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, n, Lr->b, Lr->x);
    LAUNCH_CHECK();
    for (int k = 0; k < Lr->n_unroll; ++k) {
        if (keep) {
            hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, n, Lr->x, Lr->xs + (size_t)k * n);
            LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_cnn_pack, vec_grid(), dim3(kThreads), 0, st, (long)Lr->L, ns, npx, Lr->x, Lr->scal, 1,
                           Lr->act[0]);
        LAUNCH_CHECK();
        if ((s = lcnn_forward(Lr, st))) return s;
        hipLaunchKernelGGL(k_cnn_unpack_add, vec_grid(), dim3(kThreads), 0, st, (long)Lr->L, ns, npx,
                           Lr->act[smsm_learned::kDepth], Lr->x, Lr->scal, 0, Lr->z);
        LAUNCH_CHECK();
        if ((s = laxpy(Lr, Lr->b, Lr->z, nullptr, Lr->mu, Lr->rhs, st))) return s;    // b + mu z
        hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, n, Lr->z, Lr->x);   // warm start at z
        LAUNCH_CHECK();
        if ((s = ldc_cg(Lr, Lr->rhs, Lr->x, st))) return s;
    }
    return SMSM_OK;
}

// Loss ||x - xt||^2 / ||xt||^2 (numerator and denominator in scal[8], scal[9])
// and the gradients of every parameter into grads.
smsm_status lbackward(smsm_learned* Lr, const double2* xt, hipStream_t st) {
    const long n = lvec(Lr);
    const int ns = Lr->nc / 2, npx = Lr->H * Lr->W;
    double* sc = Lr->scal;
    smsm_status s;
    if ((s = laxpy(Lr, Lr->x, xt, nullptr, -1.0, Lr->g, st))) return s;              // x - xt
    if ((s = ldot(Lr, Lr->g, Lr->g, st)) || (s = lscalar(Lr, 0, nullptr, 0.0, sc + 8, st))) return s;
    if ((s = ldot(Lr, xt, xt, st)) || (s = lscalar(Lr, 0, nullptr, 0.0, sc + 9, st))) return s;
    hipLaunchKernelGGL(k_dc_grad0, vec_grid(), dim3(kThreads), 0, st, n, Lr->g, sc + 9);   // g = 2 (x - xt) / den
    LAUNCH_CHECK();
    for (int k = Lr->n_unroll - 1; k >= 0; --k) {
        hipLaunchKernelGGL(k_zero_c128, vec_grid(), dim3(kThreads), 0, st, n, Lr->wv);
        LAUNCH_CHECK();
        if ((s = ldc_cg(Lr, Lr->g, Lr->wv, st))) return s;                          // w = M^-1 g
        if ((s = laxpy(Lr, nullptr, Lr->wv, nullptr, Lr->mu, Lr->z, st))) return s;   // gz = mu w (in z)
        hipLaunchKernelGGL(k_cnn_pack, vec_grid(), dim3(kThreads), 0, st, (long)Lr->L, ns, npx, Lr->xs + (size_t)k * n,
                           Lr->scal, 1, Lr->act[0]);
        LAUNCH_CHECK();
        if ((s = lcnn_forward(Lr, st))) return s;                                    // activations of step k
        hipLaunchKernelGGL(k_cnn_pack, vec_grid(), dim3(kThreads), 0, st, (long)Lr->L, ns, npx, Lr->z, Lr->scal, 0,
                           Lr->gio);                                                 // s (Re gz, Im gz)
        LAUNCH_CHECK();
        if ((s = lcnn_backward(Lr, Lr->gio, Lr->gio, k < Lr->n_unroll - 1 ? 1 : 0, st))) return s;
        hipLaunchKernelGGL(k_cnn_unpack_add, vec_grid(), dim3(kThreads), 0, st, (long)Lr->L, ns, npx, Lr->gio, Lr->z,
                           Lr->scal, 1, Lr->g);                                      // g = gz + gin / s
        LAUNCH_CHECK();
    }
    return SMSM_OK;
}

void learned_release(smsm_learned* Lr) {
    if (!Lr) return;
    if (Lr->arena && hipSetDevice(Lr->dev) == hipSuccess) (void)hipFree(Lr->arena);
    delete Lr;
}

}  // namespace

extern "C" {

smsm_status smsm_learned_create(smsm_plan* P, int width, int n_unroll, int n_cg, double mu, const float* params_host,
                                smsm_learned** out) {
    if (!P || !out || !params_host || n_unroll < 1 || n_cg < 1 || !(mu > 0.0) || width < 8 || width % 8 != 0 ||
        width > 256)
        return SMSM_E_INVALID;
    *out = nullptr;
    const Geo& g = P->g;
    if ((2 * g.Ns) % 4 != 0) return SMSM_E_UNSUPPORTED;    // 2 Ns channels must be a multiple of 4
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    smsm_learned* Lr = new (std::nothrow) smsm_learned;
    if (!Lr) return SMSM_E_NOMEM;
    Lr->P = P;
    Lr->dev = P->dev;
    Lr->width = width;
    Lr->nc = 2 * g.Ns;
    Lr->L = g.L;
    Lr->H = g.n2;
    Lr->W = g.n1;
    Lr->n_unroll = n_unroll;
    Lr->n_cg = n_cg;
    Lr->mu = mu;
    size_t off = 0;
    for (int k = 0; k < smsm_learned::kDepth; ++k) {
        Lr->cin[k] = k == 0 ? Lr->nc : width;
        Lr->cout[k] = k == smsm_learned::kDepth - 1 ? Lr->nc : width;
        Lr->woff[k] = off;
        off += (size_t)Lr->cout[k] * Lr->cin[k] * 9;
        Lr->boff[k] = off;
        off += Lr->cout[k];
    }
    Lr->nparam = off;
    const size_t npx = (size_t)Lr->H * Lr->W, n = (size_t)lvec(Lr);
    const size_t ny = (size_t)g.Ns * g.Nc * npx;
    Carver cv;
    const size_t oprm = cv.take<float>(off), ogr = cv.take<float>(off), oam = cv.take<float>(off),
                 oav = cv.take<float>(off);
    size_t oact[smsm_learned::kDepth + 1];
    for (int k = 0; k <= smsm_learned::kDepth; ++k)
        oact[k] = cv.take<float>((size_t)Lr->L * (k == 0 || k == smsm_learned::kDepth ? Lr->nc : width) * npx);
    const size_t oga = cv.take<float>((size_t)Lr->L * width * npx), ogb = cv.take<float>((size_t)Lr->L * width * npx);
    const size_t ogio = cv.take<float>((size_t)Lr->L * Lr->nc * npx);
    size_t ov[9];
    for (int k = 0; k < 9; ++k) ov[k] = cv.take<double2>(n);
    const size_t oax = cv.take<double2>(ny), oxs = cv.take<double2>(n * n_unroll);
    const size_t opart = cv.take<double>(kVecBlocks), oscal = cv.take<double>(16);
    const size_t opart2 = cv.take<double>(kVecBlocks);
    size_t maxcc = 0, maxco = 0;
    for (int k = 0; k < smsm_learned::kDepth; ++k) {
        maxcc = std::max(maxcc, (size_t)Lr->cin[k] * Lr->cout[k]);
        maxco = std::max(maxco, (size_t)Lr->cout[k]);
    }
    const size_t nchunk = (size_t)Lr->L * std::max(wg_chunks(Lr->H, Lr->W), wgm_chunks(Lr->H, Lr->W));
    const size_t owp = cv.take<float>(nchunk * maxcc * 9), owb = cv.take<float>(nchunk * maxco);
    size_t opk[smsm_learned::kDepth][2];
    for (int k = 0; k < smsm_learned::kDepth; ++k) {
        Lr->pk_rows[k][0] = cm_round(Lr->cout[k], 16);
        Lr->pk_cols[k][0] = cm_round(Lr->cin[k], CM_CK);
        Lr->pk_rows[k][1] = cm_round(Lr->cin[k], 16);
        Lr->pk_cols[k][1] = cm_round(Lr->cout[k], CM_CK);
        for (int d = 0; d < 2; ++d)
            opk[k][d] = cv.take<unsigned short>((size_t)Lr->pk_rows[k][d] * 9 * Lr->pk_cols[k][d]);
    }
    if (hipMalloc(&Lr->arena, cv.off) != hipSuccess) {
        delete Lr;
        return SMSM_E_NOMEM;
    }
    char* base = static_cast<char*>(Lr->arena);
    Lr->params = (float*)(base + oprm);
    Lr->grads = (float*)(base + ogr);
    Lr->am = (float*)(base + oam);
    Lr->av = (float*)(base + oav);
    for (int k = 0; k <= smsm_learned::kDepth; ++k) Lr->act[k] = (float*)(base + oact[k]);
    Lr->ga = (float*)(base + oga);
    Lr->gbuf = (float*)(base + ogb);
    Lr->gio = (float*)(base + ogio);
    double2** vecs[9] = {&Lr->b, &Lr->x, &Lr->z, &Lr->r, &Lr->p, &Lr->q, &Lr->rhs, &Lr->g, &Lr->wv};
    for (int k = 0; k < 9; ++k) *vecs[k] = (double2*)(base + ov[k]);
    Lr->ax = (double2*)(base + oax);
    Lr->xs = (double2*)(base + oxs);
    Lr->part = (double*)(base + opart);
    Lr->part2 = (double*)(base + opart2);
    Lr->scal = (double*)(base + oscal);
    Lr->wpart = (float*)(base + owp);
    Lr->wbpart = (float*)(base + owb);
    for (int k = 0; k < smsm_learned::kDepth; ++k)
        for (int d = 0; d < 2; ++d) Lr->wpk[k][d] = (unsigned short*)(base + opk[k][d]);
    bool ok = hipMemcpy(Lr->params, params_host, off * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemset(Lr->am, 0, off * sizeof(float)) == hipSuccess;
    ok = ok && hipMemset(Lr->av, 0, off * sizeof(float)) == hipSuccess;
    ok = ok && hipMemset(Lr->grads, 0, off * sizeof(float)) == hipSuccess;
    ok = ok && hipMemset(Lr->scal, 0, 16 * sizeof(double)) == hipSuccess;
    if (!ok) {
        learned_release(Lr);
        return SMSM_E_DEVICE;
    }
    *out = Lr;
    return SMSM_OK;
}

smsm_status smsm_learned_destroy(smsm_learned* Lr) {
    learned_release(Lr);
    return SMSM_OK;
}

long smsm_learned_param_count(const smsm_learned* Lr) { return Lr ? (long)Lr->nparam : 0; }

smsm_status smsm_learned_get_params(smsm_learned* Lr, float* host) {
    if (!Lr || !host) return SMSM_E_INVALID;
    if (hipSetDevice(Lr->dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return SMSM_E_DEVICE;
    return hipMemcpy(host, Lr->params, Lr->nparam * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess
               ? SMSM_OK : SMSM_E_DEVICE;
}

smsm_status smsm_learned_set_params(smsm_learned* Lr, const float* host) {
    if (!Lr || !host) return SMSM_E_INVALID;
    if (hipSetDevice(Lr->dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return SMSM_E_DEVICE;
    if (hipMemcpy(Lr->params, host, Lr->nparam * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return SMSM_E_DEVICE;
    Lr->adam_t = 0;
    const bool ok = hipMemset(Lr->am, 0, Lr->nparam * sizeof(float)) == hipSuccess &&
                    hipMemset(Lr->av, 0, Lr->nparam * sizeof(float)) == hipSuccess;
    if (!ok) return SMSM_E_DEVICE;
    smsm_status s = lrefresh_bf16(Lr, nullptr);
    if (s) return s;
    return hipDeviceSynchronize() == hipSuccess ? SMSM_OK : SMSM_E_DEVICE;
}

smsm_status smsm_learned_set_bf16(smsm_learned* Lr, int on) {
    if (!Lr || on < 0 || on > 2) return SMSM_E_INVALID;
    if (hipSetDevice(Lr->dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return SMSM_E_DEVICE;
    Lr->bf16 = on;
    smsm_status s = lrefresh_bf16(Lr, nullptr);
    if (s) return s;
    return hipDeviceSynchronize() == hipSuccess ? SMSM_OK : SMSM_E_DEVICE;
}

smsm_status smsm_learned_cnn_forward(smsm_learned* Lr, const void* in_dev, void* out_dev, void* stream) {
    if (!Lr || !in_dev || !out_dev) return SMSM_E_INVALID;
    if (hipSetDevice(Lr->dev) != hipSuccess) return SMSM_E_DEVICE;
    hipStream_t st = S(stream);
    const size_t bytes = (size_t)Lr->L * Lr->nc * Lr->H * Lr->W * sizeof(float);
    if (hipMemcpyAsync(Lr->act[0], in_dev, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return SMSM_E_DEVICE;
    smsm_status s = lcnn_forward(Lr, st);
    if (s) return s;
    return hipMemcpyAsync(out_dev, Lr->act[smsm_learned::kDepth], bytes, hipMemcpyDeviceToDevice, st) == hipSuccess
               ? SMSM_OK : SMSM_E_DEVICE;
}

smsm_status smsm_learned_cnn_backward(smsm_learned* Lr, const void* in_dev, const void* gout_dev, void* gin_dev,
                                      float* grads_host, void* stream) {
    if (!Lr || !in_dev || !gout_dev || !gin_dev || !grads_host) return SMSM_E_INVALID;
    if (hipSetDevice(Lr->dev) != hipSuccess) return SMSM_E_DEVICE;
    hipStream_t st = S(stream);
    const size_t bytes = (size_t)Lr->L * Lr->nc * Lr->H * Lr->W * sizeof(float);
    if (hipMemcpyAsync(Lr->act[0], in_dev, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return SMSM_E_DEVICE;
    smsm_status s = lcnn_forward(Lr, st);
    if (s) return s;
    if (hipMemcpyAsync(Lr->gio, gout_dev, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return SMSM_E_DEVICE;
    if ((s = lcnn_backward(Lr, Lr->gio, Lr->gio, 0, st))) return s;
    if (hipMemcpyAsync(gin_dev, Lr->gio, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return SMSM_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return SMSM_E_DEVICE;
    return hipMemcpy(grads_host, Lr->grads, Lr->nparam * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess
               ? SMSM_OK : SMSM_E_DEVICE;
}

smsm_status smsm_learned_solve(smsm_learned* Lr, const void* y_dev, void* x_dev, void* stream) {
    if (!Lr || !y_dev || !x_dev) return SMSM_E_INVALID;
    if (!Lr->P->ws) return SMSM_E_INVALID;   // the plan's workspace carries the CG vectors
    if (hipSetDevice(Lr->dev) != hipSuccess) return SMSM_E_DEVICE;
    hipStream_t st = S(stream);
    smsm_status s = lsetup(Lr, y_dev, st);
    if (s) return s;
    if ((s = lforward(Lr, false, st))) return s;
    hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, lvec(Lr), Lr->x, (double2*)x_dev);
    LAUNCH_CHECK();
    return SMSM_OK;
}

smsm_status smsm_learned_gradients(smsm_learned* Lr, const void* y_dev, const void* xt_dev, double* loss,
                                   float* grads_host, void* stream) {
    if (!Lr || !y_dev || !xt_dev || !loss) return SMSM_E_INVALID;
    if (!Lr->P->ws) return SMSM_E_INVALID;   // the plan's workspace carries the CG vectors
    if (hipSetDevice(Lr->dev) != hipSuccess) return SMSM_E_DEVICE;
    hipStream_t st = S(stream);
    smsm_status s = lsetup(Lr, y_dev, st);
    if (s) return s;
    if ((s = lforward(Lr, true, st))) return s;
    if ((s = lbackward(Lr, (const double2*)xt_dev, st))) return s;
    double nd[2];
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(nd, Lr->scal + 8, 2 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return SMSM_E_DEVICE;
    *loss = nd[1] > 0.0 ? nd[0] / nd[1] : 0.0;
    if (grads_host &&
        hipMemcpy(grads_host, Lr->grads, Lr->nparam * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return SMSM_E_DEVICE;
    return SMSM_OK;
}

smsm_status smsm_learned_train_step(smsm_learned* Lr, const void* y_dev, const void* xt_dev, double lr,
                                    double* loss, void* stream) {
    if (!Lr || !(lr > 0.0)) return SMSM_E_INVALID;
    smsm_status s = smsm_learned_gradients(Lr, y_dev, xt_dev, loss, nullptr, stream);
    if (s) return s;
    ++Lr->adam_t;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - (float)std::pow(0.9, (double)Lr->adam_t), c2 = 1.0f - (float)std::pow(0.999, (double)Lr->adam_t);
    hipLaunchKernelGGL(k_adam, vec_grid(), dim3(kThreads), 0, S(stream), (long)Lr->nparam, Lr->params, Lr->grads,
                       Lr->am, Lr->av, (float)lr, b1, b2, 1e-8f, c1, c2);
    LAUNCH_CHECK();
    return lrefresh_bf16(Lr, S(stream));
}

// The plain IRLS solve of y into the object's vector wv (complex128 output
// for that call whatever the plan's output flag).
static smsm_status plain_into(smsm_learned* Lr, const void* y_dev, void* stream) {
    smsm_plan* P = Lr->P;
    const uint32_t flags = P->prm.flags;
    P->prm.flags = flags | SMSM_FLAG_X_C128;
    const smsm_status s = smsm_solve(P, y_dev, Lr->wv, stream);
    P->prm.flags = flags;
    return s;
}

smsm_status smsm_learned_solve_fallback(smsm_learned* Lr, const void* y_dev, void* x_dev, double ratio,
                                        double res_ref, double* res_out, int* fell_back, void* stream) {
    if (!Lr || !y_dev || !x_dev || !res_out || !fell_back || !(ratio > 0.0)) return SMSM_E_INVALID;
    smsm_status s = smsm_learned_solve(Lr, y_dev, x_dev, stream);
    if (s) return s;
    double r_l = 0.0, r_p = res_ref;
    if ((s = smsm_learned_residual(Lr, x_dev, y_dev, &r_l, stream))) return s;
    bool have_plain = false;
    if (!(r_p > 0.0)) {
        if ((s = plain_into(Lr, y_dev, stream))) return s;
        if ((s = smsm_learned_residual(Lr, Lr->wv, y_dev, &r_p, stream))) return s;
        have_plain = true;
    }
    *fell_back = r_l > ratio * r_p ? 1 : 0;
    if (*fell_back) {
        if (!have_plain && (s = plain_into(Lr, y_dev, stream))) return s;
        hipStream_t st = S(stream);
        hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, lvec(Lr), Lr->wv, (double2*)x_dev);
        LAUNCH_CHECK();
        if (hipStreamSynchronize(st) != hipSuccess) return SMSM_E_DEVICE;
    }
    res_out[0] = r_l;
    res_out[1] = r_p;
    return SMSM_OK;
}

smsm_status smsm_learned_residual(smsm_learned* Lr, const void* x_dev, const void* y_dev, double* res, void* stream) {
    if (!Lr || !x_dev || !y_dev || !res) return SMSM_E_INVALID;
    hipStream_t st = S(stream);
    smsm_status s = smsm_apply_A(Lr->P, x_dev, Lr->ax, stream);
    if (s) return s;
    const Geo& g = Lr->P->g;
    const long ny = (long)g.Ns * g.Nc * g.n2 * g.n1;
    hipLaunchKernelGGL(k_dc_resid, vec_grid(), dim3(kThreads), 0, st, ny, Lr->ax, (const float2*)y_dev, Lr->part);
    LAUNCH_CHECK();
    if ((s = lscalar(Lr, 0, nullptr, 0.0, Lr->scal + 10, st))) return s;
    double v = 0.0;
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(&v, Lr->scal + 10, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return SMSM_E_DEVICE;
    *res = std::sqrt(v);
    return SMSM_OK;
}

}  // extern "C"

// ---- augmented-Lagrangian solve ------------------------------------------

struct smsm_al {
    smsm_plan* P = nullptr;
    int dev = 0;
    AlGeo a{};
    double lam = 0.0, beta = 0.0, tau = 0.0;
    int n_outer = 0, n_cg = 0, n_sign = 0, nit_w = 0;
    uint32_t flags = 0;
    int chunk = 0, nchunk = 0, ntile = 0, npmax = 0;
    void* arena = nullptr;
    size_t bytes = 0;
    double2 *b = nullptr, *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *rhs = nullptr;
    double2 *hzu = nullptr, *hu = nullptr;   // H^H(Z - U) and H^H(U), [L][Ns][n2][n1]
    double2* U[2] = {};                      // scaled duals [L][K][NPP]; U[cur] after a solve
    int cur = 0;
    double2* gpart = nullptr;                // Gram partials [L][nchunk][pairs][64][64]
    double2 *G = nullptr, *Q = nullptr, *X[2] = {}, *T = nullptr, *Pr = nullptr, *C = nullptr;
    double2 *Y[2] = {}, *Z[2] = {}, *Wp = nullptr, *F = nullptr;   // [L][KP][KP]
    double *dpart0 = nullptr, *dpart1 = nullptr;   // dense partials [L][npmax]
    double* smu = nullptr;    // mu^2 of the sign iteration's steps
    double* ones = nullptr;   // [L] ones (unscaled products)
    int* zeros = nullptr;     // [L] zeros (never-converged flags of the sign steps)
    double *nsmu = nullptr, *wscale = nullptr, *tau2 = nullptr;
    int* done = nullptr;      // coupled iteration: [(nit_w + 2) L]
    double *part = nullptr, *scal = nullptr;   // CG partials [kVecBlocks], scalars
};

namespace {

constexpr int kAlChunks = 64;          // patch chunks of the Gram partials
constexpr int kAlUpdWaves = 8;         // dual update: waves (16 rows of K each) per workgroup
constexpr double kAlSignLo = 1e-14;    // sign iteration: resolution relative to ||G - tau^2 I||_F
constexpr double kAlMuMax = 1.6;       // largest scale of a sign step (p(1.6) = 0.352 > 0)
constexpr int kAlNsIters = 30;         // cap of the coupled iteration for Gt^(-1/2)

// Scales mu_k of the sign iteration X <- p(mu_k X), p(t) = 1.5 t - 0.5 t^3,
// for a spectrum |X| within [lo, 1]: mu maximises the lower end, min(p(mu lo),
// p(mu)) (p is increasing up to 1 and decreasing beyond), capped at
// kAlMuMax; then plain steps until the lower end is 1 to rounding, and one
// more.  The upper end stays 1 (p(mu t) peaks at t = 1/mu with value 1).
std::vector<double> al_sign_schedule(double lo) {
    auto pf = [](double t) { return 1.5 * t - 0.5 * t * t * t; };
    std::vector<double> mu;
    while (1.0 - lo > 1e-16 && mu.size() < 200) {
        double m = 1.0;
        if (lo < 0.5) {
            if (pf(kAlMuMax * lo) < pf(kAlMuMax)) {
                m = kAlMuMax;
            } else {
                double u = 1.0, v = kAlMuMax;
                for (int it = 0; it < 80; ++it) {
                    const double c = 0.5 * (u + v);
                    if (pf(c * lo) < pf(c)) u = c;
                    else v = c;
                }
                m = 0.5 * (u + v);
            }
        }
        lo = std::min(pf(m * lo), pf(m));
        mu.push_back(m);
    }
    mu.push_back(1.0);
    return mu;
}

smsm_status al_launch_gemm_norm(smsm_al* A, const double2* a0, const double2* b0, double2* c0, hipStream_t st) {
    HgArgs u{};
    u.A0 = a0; u.B0 = b0; u.C0 = c0;
    u.part_in = A->ones;
    u.np_in = 1;
    u.part_out = A->dpart1;
    hipLaunchKernelGGL(k_zgemm<HG_NORM>, dim3(A->ntile, 1, A->a.L), dim3(64 * HW), 0, st, A->a.K, A->a.KP, u);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// F = f(M^H M) of the split M = H(x) + U[cur] (see smsm_al.h).
smsm_status al_threshold(smsm_al* A, hipStream_t st) {
    const AlGeo& a = A->a;
    const int npair = a.KB * (a.KB + 1) / 2;
    hipLaunchKernelGGL(k_al_gram, dim3(npair, A->nchunk, a.L), dim3(kThreads), 0, st, a, A->x, A->U[A->cur],
                       A->chunk, A->gpart);
    LAUNCH_CHECK();
    const dim3 dg(kPadBlocks, a.L);
    hipLaunchKernelGGL(k_al_gram_sum, dg, dim3(kThreads), 0, st, a, A->gpart, A->nchunk, A->tau * A->tau, A->G,
                       A->Q, A->dpart0);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_al_sign_start, dg, dim3(kThreads), 0, st, a.KP, A->Q, A->dpart0, kPadBlocks, A->X[0]);
    LAUNCH_CHECK();
    int xc = 0;
    for (int k = 0; k < A->n_sign; ++k) {
        HgArgs t{};
        t.A0 = A->X[xc]; t.B0 = A->X[xc]; t.C0 = A->T;
        t.done_cur = A->zeros;
        t.part_out = A->dpart0;
        t.mu = A->smu + k;
        t.mu_stride = 0;
        hipLaunchKernelGGL(k_zgemm<HG_NS>, dim3(A->ntile, 1, a.L), dim3(64 * HW), 0, st, a.K, a.KP, t);
        LAUNCH_CHECK();
        smsm_status s = al_launch_gemm_norm(A, A->X[xc], A->T, A->X[xc ^ 1], st);
        if (s) return s;
        xc ^= 1;
    }
    hipLaunchKernelGGL(k_al_proj, dg, dim3(kThreads), 0, st, a.K, a.KP, A->X[xc], A->Pr);
    LAUNCH_CHECK();
    smsm_status s = al_launch_gemm_norm(A, A->G, A->Pr, A->C, st);
    if (s) return s;
    hipLaunchKernelGGL(k_al_gtilde, dg, dim3(kThreads), 0, st, a.K, a.KP, A->C, A->Pr, A->tau * A->tau, A->Y[0],
                       A->dpart0);
    LAUNCH_CHECK();
    const int nit = A->nit_w;
    hipLaunchKernelGGL(k_ns_start, dg, dim3(kThreads), 0, st, a.K, a.KP, a.L, A->tau2, 1.0, A->dpart0, kPadBlocks,
                       A->Y[0], A->Z[0], A->wscale, A->done, nit, A->nsmu);
    LAUNCH_CHECK();
    for (int k = 0; k < nit; ++k) {
        const int c0 = k & 1, c1 = c0 ^ 1;
        HgArgs t{};
        t.A0 = A->Z[c0]; t.B0 = A->Y[c0]; t.C0 = A->T;
        t.done_cur = A->done + (size_t)k * a.L;
        t.part_out = A->dpart0;
        t.mu = A->nsmu + (size_t)k * a.L;
        t.mu_stride = 1;
        hipLaunchKernelGGL(k_zgemm<HG_NS>, dim3(A->ntile, 1, a.L), dim3(64 * HW), 0, st, a.K, a.KP, t);
        LAUNCH_CHECK();
        HgArgs u{};
        u.A0 = A->Y[c0]; u.B0 = A->T; u.C0 = A->Y[c1];
        u.A1 = A->T; u.B1 = A->Z[c0]; u.C1 = A->Z[c1];
        u.done_cur = A->done + (size_t)k * a.L;
        u.done_next = A->done + (size_t)(k + 1) * a.L;
        u.last = A->done + (size_t)(nit + 1) * a.L;
        u.par = c1;
        u.tol2 = kNsTol * kNsTol;
        u.part_in = A->dpart0;
        u.np_in = A->ntile;
        hipLaunchKernelGGL(k_zgemm<HG_PAIR>, dim3(A->ntile, 1, 2 * a.L), dim3(64 * HW), 0, st, a.K, a.KP, u);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_al_pick, dg, dim3(kThreads), 0, st, a.K, a.KP, A->Z[0], A->Z[1],
                       A->done + (size_t)(nit + 1) * a.L, A->done + (size_t)nit * a.L, A->wscale, A->Wp,
                       A->P->flags);
    LAUNCH_CHECK();
    if ((s = al_launch_gemm_norm(A, A->Pr, A->Wp, A->C, st))) return s;
    hipLaunchKernelGGL(k_al_f, dg, dim3(kThreads), 0, st, a.K, a.KP, A->C, A->Pr, A->tau, A->F);
    LAUNCH_CHECK();
    return SMSM_OK;
}

long al_nvec(const smsm_al* A) { return (long)A->a.L * A->a.Ns * A->a.n2 * A->a.n1; }

smsm_status al_dot(smsm_al* A, const double2* u, const double2* v, hipStream_t st) {
    hipLaunchKernelGGL(k_dc_dot, vec_grid(), dim3(kThreads), 0, st, al_nvec(A), u, v, A->part);
    LAUNCH_CHECK();
    return SMSM_OK;
}
smsm_status al_scalar(smsm_al* A, int mode, double* rr, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_dc_scalar, dim3(1), dim3(kThreads), 0, st, mode, A->part, kVecBlocks, rr, 0.0, out);
    LAUNCH_CHECK();
    return SMSM_OK;
}
smsm_status al_axpy(smsm_al* A, const double2* u, const double2* v, const double* fp, double fm, double2* out,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_dc_axpy, vec_grid(), dim3(kThreads), 0, st, al_nvec(A), u, v, fp, fm, out);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// out = (A^H A + (beta/2) c) v
smsm_status al_normal(smsm_al* A, const double2* v, double2* out, hipStream_t st) {
    smsm_status s = chain_normal(A->P, v, out, COL_NORMAL, false, st);
    if (s) return s;
    hipLaunchKernelGGL(k_al_diag, vec_grid(), dim3(kThreads), 0, st, A->a, v, 0.5 * A->beta, out);
    LAUNCH_CHECK();
    return SMSM_OK;
}

// n_cg CG steps on the x-step's system from the current x (the oracle's
// recurrence: r = rhs - N x, p = r, alpha = |r|^2 / <p, N p>, beta = |r'|^2 / |r|^2).
smsm_status al_cg(smsm_al* A, hipStream_t st) {
    double* sc = A->scal;
    smsm_status s;
    if ((s = al_normal(A, A->x, A->q, st))) return s;
    if ((s = al_axpy(A, A->rhs, A->q, nullptr, -1.0, A->r, st))) return s;
    hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, al_nvec(A), A->r, A->p);
    LAUNCH_CHECK();
    if ((s = al_dot(A, A->r, A->r, st)) || (s = al_scalar(A, 0, nullptr, sc + 1, st))) return s;
    for (int j = 0; j < A->n_cg; ++j) {
        if ((s = al_normal(A, A->p, A->q, st))) return s;
        if ((s = al_dot(A, A->p, A->q, st)) || (s = al_scalar(A, 1, sc + 1, sc + 2, st))) return s;
        if ((s = al_axpy(A, A->x, A->p, sc + 2, 1.0, A->x, st))) return s;
        if ((s = al_axpy(A, A->r, A->q, sc + 2, -1.0, A->r, st))) return s;
        if ((s = al_dot(A, A->r, A->r, st)) || (s = al_scalar(A, 2, sc + 1, sc + 3, st))) return s;
        if ((s = al_axpy(A, A->r, A->p, sc + 3, 1.0, A->p, st))) return s;
    }
    return SMSM_OK;
}

void al_release(smsm_al* A) {
    if (!A) return;
    if (A->arena && hipSetDevice(A->dev) == hipSuccess) (void)hipFree(A->arena);
    delete A;
}

}  // namespace

extern "C" {

smsm_status smsm_al_create(smsm_plan* P, const smsm_al_params* prm, smsm_al** out) {
    if (!out) return SMSM_E_INVALID;
    *out = nullptr;
    if (!P || !prm || !(prm->lambda > 0.0) || !(prm->beta > 0.0) || prm->n_outer < 1 || prm->n_cg < 0 ||
        prm->n_sign < 0 || prm->n_sign > 200 || (prm->flags & ~SMSM_FLAG_X_C128))
        return SMSM_E_INVALID;
    if (hipSetDevice(P->dev) != hipSuccess) return SMSM_E_DEVICE;
    const Geo& g = P->g;
    smsm_al* A = new (std::nothrow) smsm_al;
    if (!A) return SMSM_E_NOMEM;
    A->P = P;
    A->dev = P->dev;
    AlGeo& a = A->a;
    a.n1 = g.n1; a.n2 = g.n2; a.L = g.L; a.Ns = g.Ns; a.r = g.r; a.K = g.K; a.KP = dense_stride(g.K);
    a.P1 = g.n1 - g.r + 1; a.P2 = g.n2 - g.r + 1; a.NP = a.P1 * a.P2;
    a.NPP = (a.NP + AL_PT - 1) / AL_PT * AL_PT;
    a.KB = (g.K + AL_BK - 1) / AL_BK;
    A->lam = prm->lambda;
    A->beta = prm->beta;
    A->tau = prm->lambda / prm->beta;
    A->n_outer = prm->n_outer;
    A->n_cg = prm->n_cg;
    A->flags = prm->flags;
    A->nit_w = kAlNsIters;
    std::vector<double> smu = al_sign_schedule(kAlSignLo);
    if (prm->n_sign > 0) smu.resize(prm->n_sign, 1.0);
    A->n_sign = (int)smu.size();
    for (double& m : smu) m = m * m;   // k_zgemm<HG_NS> takes mu^2 (its T = sqrt(m) (1.5 I - 0.5 m X^2))
    A->nchunk = std::min(kAlChunks, (a.NP + AL_SL - 1) / AL_SL);
    A->chunk = ((a.NP + A->nchunk - 1) / A->nchunk + AL_SL - 1) / AL_SL * AL_SL;
    A->nchunk = (a.NP + A->chunk - 1) / A->chunk;
    A->ntile = dense_tiles(g.K);
    A->npmax = std::max(A->ntile, kPadBlocks);
    const size_t nvec = (size_t)g.L * g.Ns * g.n2 * g.n1;
    const size_t nu = (size_t)g.L * g.K * a.NPP;
    const size_t nd = (size_t)g.L * a.KP * a.KP;
    const int npair = a.KB * (a.KB + 1) / 2;
    Carver cv;
    size_t ov[8];
    for (int k = 0; k < 8; ++k) ov[k] = cv.take<double2>(nvec);
    const size_t ou0 = cv.take<double2>(nu), ou1 = cv.take<double2>(nu);
    const size_t ogp = cv.take<double2>((size_t)g.L * A->nchunk * npair * AL_BK * AL_BK);
    size_t od[13];
    for (int k = 0; k < 13; ++k) od[k] = cv.take<double2>(nd);
    const size_t op0 = cv.take<double>((size_t)g.L * A->npmax), op1 = cv.take<double>((size_t)g.L * A->npmax);
    const size_t osmu = cv.take<double>(smu.size()), oones = cv.take<double>(g.L), ozeros = cv.take<int>(g.L);
    const size_t onsmu = cv.take<double>((size_t)A->nit_w * g.L), ows = cv.take<double>(g.L),
                 otau2 = cv.take<double>(g.L);
    const size_t odone = cv.take<int>((size_t)(A->nit_w + 2) * g.L);
    const size_t opart = cv.take<double>(kVecBlocks), oscal = cv.take<double>(16);
    A->bytes = cv.off;
    if (hipMalloc(&A->arena, cv.off) != hipSuccess) {
        delete A;
        return SMSM_E_NOMEM;
    }
    char* base = static_cast<char*>(A->arena);
    double2** vecs[8] = {&A->b, &A->x, &A->r, &A->p, &A->q, &A->rhs, &A->hzu, &A->hu};
    for (int k = 0; k < 8; ++k) *vecs[k] = (double2*)(base + ov[k]);
    A->U[0] = (double2*)(base + ou0);
    A->U[1] = (double2*)(base + ou1);
    A->gpart = (double2*)(base + ogp);
    double2** dn[13] = {&A->G, &A->Q, &A->X[0], &A->X[1], &A->T, &A->Pr, &A->C,
                        &A->Y[0], &A->Y[1], &A->Z[0], &A->Z[1], &A->Wp, &A->F};
    for (int k = 0; k < 13; ++k) *dn[k] = (double2*)(base + od[k]);
    A->dpart0 = (double*)(base + op0);
    A->dpart1 = (double*)(base + op1);
    A->smu = (double*)(base + osmu);
    A->ones = (double*)(base + oones);
    A->zeros = (int*)(base + ozeros);
    A->nsmu = (double*)(base + onsmu);
    A->wscale = (double*)(base + ows);
    A->tau2 = (double*)(base + otau2);
    A->done = (int*)(base + odone);
    A->part = (double*)(base + opart);
    A->scal = (double*)(base + oscal);
    std::vector<double> ones(g.L, 1.0), t2(g.L, A->tau * A->tau);
    std::vector<int> zeros(g.L, 0);
    bool ok = hipMemcpy(A->smu, smu.data(), smu.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(A->ones, ones.data(), g.L * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(A->zeros, zeros.data(), g.L * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(A->tau2, t2.data(), g.L * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    // the dense buffers' padding stays zero from here on (every kernel writes zeros there)
    ok = ok && hipMemset(base + ov[0], 0, osmu - ov[0]) == hipSuccess;
    ok = ok && hipMemset(A->scal, 0, 16 * sizeof(double)) == hipSuccess;
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        al_release(A);
        return SMSM_E_DEVICE;
    }
    *out = A;
    return SMSM_OK;
}

smsm_status smsm_al_destroy(smsm_al* A) {
    if (A && hipSetDevice(A->dev) == hipSuccess) (void)hipDeviceSynchronize();
    al_release(A);
    return SMSM_OK;
}

size_t smsm_al_device_bytes(const smsm_al* A) { return A ? A->bytes : 0; }

smsm_status smsm_al_solve(smsm_al* A, const void* y_dev, void* x_dev, void* stream) {
    if (!A || !y_dev || !x_dev) return SMSM_E_INVALID;
    smsm_plan* P = A->P;
    if (!P->ws) return SMSM_E_INVALID;   // the plan's workspace carries the operator chains' buffers
    if (hipSetDevice(A->dev) != hipSuccess) return SMSM_E_DEVICE;
    hipStream_t st = S(stream);
    const AlGeo& a = A->a;
    const long n = al_nvec(A);
    smsm_status s = chain_AH_hyb(P, (const float2*)y_dev, P->h2, st);
    if (s) return s;
    if ((s = rows_fwd(P, P->h2, A->b, st))) return s;                          // b = A^H y
    hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, n, A->b, A->x);   // x0 = b
    LAUNCH_CHECK();
    A->cur = 0;
    hipLaunchKernelGGL(k_zero_c128, vec_grid(), dim3(kThreads), 0, st, (long)a.L * a.K * a.NPP, A->U[0]);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_al_init, vec_grid(), dim3(kThreads), 0, st, a, A->x, A->hu, A->hzu);
    LAUNCH_CHECK();
    const int kbu = (a.K + 16 * kAlUpdWaves - 1) / (16 * kAlUpdWaves);
    for (int it = 0; it < A->n_outer; ++it) {
        if ((s = al_axpy(A, A->b, A->hzu, nullptr, 0.5 * A->beta, A->rhs, st))) return s;   // b + (beta/2) H^H(Z - U)
        if ((s = al_cg(A, st))) return s;
        if ((s = al_threshold(A, st))) return s;
        hipLaunchKernelGGL(k_al_update<kAlUpdWaves>, dim3(a.NPP / AL_PT * kbu, 1, a.L), dim3(64 * kAlUpdWaves), 0,
                           st, a, A->x, A->U[A->cur], A->F, A->U[A->cur ^ 1]);
        LAUNCH_CHECK();
        A->cur ^= 1;
        hipLaunchKernelGGL(k_al_gather, dim3(1024), dim3(kThreads), 0, st, a, A->x, A->U[A->cur], A->hu, A->hzu);
        LAUNCH_CHECK();
    }
    if (A->flags & SMSM_FLAG_X_C128)
        hipLaunchKernelGGL(k_copy_c128, vec_grid(), dim3(kThreads), 0, st, n, A->x, (double2*)x_dev);
    else
        hipLaunchKernelGGL(k_to_c64, vec_grid(), dim3(kThreads), 0, st, n, A->x, (float2*)x_dev);
    LAUNCH_CHECK();
    return SMSM_OK;
}

smsm_status smsm_al_dual(smsm_al* A, void* u_dev, void* stream) {
    if (!A || !u_dev) return SMSM_E_INVALID;
    if (hipSetDevice(A->dev) != hipSuccess) return SMSM_E_DEVICE;
    const AlGeo& a = A->a;
    return hipMemcpyAsync(u_dev, A->U[A->cur], (size_t)a.L * a.K * a.NPP * sizeof(double2), hipMemcpyDeviceToDevice,
                          S(stream)) == hipSuccess ? SMSM_OK : SMSM_E_DEVICE;
}

long smsm_al_dual_stride(const smsm_al* A) { return A ? (long)A->a.NPP : 0; }

}  // extern "C"

