// 3 x 3 convolutions of the learned prior on the BF16 matrix cores (gfx950
// v_mfma_f32_16x16x32_bf16), BF16 weights and FP32 accumulation, in two
// forms: exact products (FP32 activations split into three BF16 parts,
// x = hi + mid + lo exact to ~2^-27 of x, so each product w x is formed to
// FP32 accuracy from three BF16 products), or the BF16 network (every
// convolution input rounded to BF16: one product).
//
// Implicit GEMM: out[o][p] = bias[o] + sum_{t, c} W[o][t][c] in[c][p + off_t].
// A workgroup (4 waves) takes an output tile of CM_TR rows x CM_TC columns of
// one image and 16 NOB output channels; wave w takes tile row w (CM_TC = 64
// pixels = 4 blocks of 16).  The input tile with its one-pixel halo is staged
// in shared memory in chunks of CM_CK = 16 channels as BF16 planes,
// position-major with the channels contiguous (16-byte fragment reads; the
// position stride of 24 BF16 puts the 16 lanes of a fragment read on
// distinct banks), and the chunk's weights (16 NOB rows of 9 taps x 16
// channels, row stride 152 BF16, again bank-distinct for a fragment read)
// beside it.  One MFMA step (K = 32) covers two taps of the chunk:
// lane group g = l / 16 takes tap 2 s + g / 2 and channels 8 (g % 2) .. + 7,
// so the 9 taps take 5 steps (the tenth tap has zero weights).  Per step a
// wave reads its weight fragments (16 bytes per lane per 16-channel block),
// then per pixel block the planes' fragments, and issues one MFMA per plane
// and output-channel block.  MFMA operand layout (16x16x32): lane l
// holds A[m = l % 16][k = 8 (l / 16) + j] and B[k = 8 (l / 16) + j][n = l % 16],
// j < 8, and receives C[m = 4 (l / 16) + j][n = l % 16], j < 4.  The sums run
// in a fixed order (chunks, steps, planes), so results are deterministic.
#pragma once
#include "smsm_device.h"

typedef __bf16 cm_bf16x8 __attribute__((ext_vector_type(8)));
typedef float cm_f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned cm_u32x4 __attribute__((ext_vector_type(4)));

#define CM_TR 4                                   // output rows per workgroup (one per wave)
#define CM_TC 64                                  // output columns per workgroup
#define CM_CK 16                                  // input channels per staged chunk
#define CM_PSTR 24                                // BF16 per staged position (16 channels + 8 spread)
#define CM_POS ((CM_TR + 2) * (CM_TC + 2))        // staged positions (tile and halo)
#define CM_WSTR (9 * CM_CK + 8)                   // BF16 per staged weight row (9 taps x 16 channels + 8 spread)

SMSM_HD inline int cm_round(int v, int m) { return (v + m - 1) / m * m; }

// BF16 bits of an FP32 value, round to nearest, ties to even.
SMSM_DEV unsigned cm_bf16_bits(float v) {
    const unsigned b = __float_as_uint(v);
    return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}
// The same for two values at once, packed (x in the low half): the gfx950
// packed conversion, one instruction (equal to cm_bf16_bits for finite values).
typedef float cm_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 cm_bf16x2 __attribute__((ext_vector_type(2)));
SMSM_DEV unsigned cm_bf16x2_bits(cm_f32x2 v) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, cm_bf16x2));
}

// Packed BF16 weights of one layer (w [co][ci][3][3], FP32) for
//   fwd (bwd = 0): P[o][t][c] = w[o][c][t],      o < rows = co rounded up to 16, c < cols = ci rounded up to 16;
//   bwd-data (1):  P[c][t][o] = w[o][c][8 - t],  c < rows = ci rounded up to 16, o < cols = co rounded up to 16;
// zero in the padding.  The BF16 rounding is that of the network's BF16 copy.
__global__ void k_conv_wpack(int ci, int co, const float* __restrict__ w, int bwd, int rows, int cols,
                             unsigned short* __restrict__ P) {
    const long total = (long)rows * 9 * cols;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const int col = (int)(k % cols);
        const long rt = k / cols;
        const int t = (int)(rt % 9), row = (int)(rt / 9);
        const int o = bwd ? col : row, c = bwd ? row : col;
        float v = 0.0f;
        if (o < co && c < ci) v = w[((size_t)o * ci + c) * 9 + (bwd ? 8 - t : t)];
        P[k] = (unsigned short)cm_bf16_bits(v);
    }
}

// One convolution (forward with packed fwd weights, or the backward-data
// transpose with packed bwd weights and no bias): ci input channels, co
// output channels, `cols` = ci rounded up to 16 (the packed row length),
// images [N][ci][H][W] -> [N][co][H][W].  PLANES = 3: the input in three BF16
// parts (products exact to FP32); PLANES = 1: the input rounded to BF16 (the
// BF16 network), and round_out != 0 stores each output rounded to a BF16
// value (the network's hidden activations).  grid (ceil(H / CM_TR)
// ceil(W / CM_TC), rows / (16 NOB), N), block 256.
//
// Workgroup order: the hardware hands consecutive workgroups to the eight
// XCDs in turn, so the logical tile of a workgroup is taken XCD-major (when
// the grid divides by eight): each XCD works through a contiguous run of
// tiles, whose shared halo rows then meet in that XCD's L2.  The output
// tile goes out through shared memory (16 channels at a time per wave), so
// that every store instruction writes whole 128-byte lines.
#define CM_EST 80    // floats per staged output channel row (64 pixels + 16: the 4 row groups of a write on distinct banks)
template <int NOB, int PLANES>
__global__ void __launch_bounds__(256, 3)
k_conv3x3_mfma(int ci, int co, int cols, int H, int W, const float* __restrict__ in,
               const unsigned short* __restrict__ P, const float* __restrict__ bias, float* __restrict__ out,
               int relu, int round_out) {
    constexpr int XS = CM_POS * CM_PSTR;     // BF16 per staged plane
    static_assert((PLANES * XS + 16 * NOB * CM_WSTR) * sizeof(unsigned short) >= 4 * 16 * CM_EST * sizeof(float),
                  "output staging fits the operand buffers");
    __shared__ __attribute__((aligned(16))) unsigned short sbuf[PLANES * XS + 16 * NOB * CM_WSTR];
    unsigned short* wsm = sbuf + PLANES * XS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, l16 = lane & 15;
    int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    {
        const int nx = gridDim.x, ny = gridDim.y, nb = nx * ny * gridDim.z;
        if ((nb & 7) == 0) {
            const int b = bx + nx * (by + ny * bz), lg = (b & 7) * (nb >> 3) + (b >> 3);
            bx = lg % nx;
            by = (lg / nx) % ny;
            bz = lg / (nx * ny);
        }
    }
    const int tiles_x = (W + CM_TC - 1) / CM_TC;
    const int ty = bx / tiles_x, tx = bx - ty * tiles_x;
    const int r0 = ty * CM_TR, c0 = tx * CM_TC, n = bz;
    const int o0 = by * 16 * NOB;
    const size_t npx = (size_t)H * W;
    const float* src = in + (size_t)n * ci * npx;
    const int half = (g & 1) * 8;               // this lane group's channels within the chunk

    cm_f32x4 acc[NOB][4];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) acc[ob][pb] = cm_f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // staging items of this thread: (channel octet, position), positions
    // consecutive across lanes; their addresses are the same for every chunk.
    // The raw values of the next chunk are loaded while the current chunk's
    // products run.
    constexpr int NIT = (CM_POS * (CM_CK / 8) + 255) / 256;
    int s_off[NIT];      // element offset of the item's first channel at chunk 0 (-1: zero or none)
    int s_lds[NIT];      // its shared-memory slot (-1: none)
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
        const int item = tid + 256 * u;
        const int oc = item / CM_POS, pos = item - oc * CM_POS;
        const int pr = pos / (CM_TC + 2), pc = pos - pr * (CM_TC + 2);
        const int i = r0 - 1 + pr, j = c0 - 1 + pc;
        const bool live = item < CM_POS * (CM_CK / 8);
        const bool inside = live && i >= 0 && i < H && j >= 0 && j < W;
        s_off[u] = inside ? (int)((size_t)oc * 8 * npx + (size_t)i * W + j) : -1;
        s_lds[u] = live ? pos * CM_PSTR + oc * 8 : -1;
    }
    float raw[NIT][8];
    auto load_chunk = [&](int cc) {
#pragma unroll
        for (int u = 0; u < NIT; ++u) {
            const int c8 = cc + (s_lds[u] >= 0 ? (s_lds[u] % CM_PSTR) : 0);   // first channel of the octet
#pragma unroll
            for (int q = 0; q < 8; ++q)
                raw[u][q] = (s_off[u] >= 0 && c8 + q < ci) ? src[(size_t)s_off[u] + (size_t)(cc + q) * npx] : 0.0f;
        }
    };
    // the chunk's weights: rows o0 .. o0 + 16 NOB - 1, 9 taps x 16 channels
    // each, 16 bytes per item
    constexpr int NW = (16 * NOB * 9 * 2 + 255) / 256;
    cm_u32x4 wraw[NW];   // (a native vector: a uint4 struct array is copied as an aggregate and stays in memory)
    auto load_weights = [&](int cc) {
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int item = tid + 256 * u;
            const int row = item / 18, rem = item - row * 18;
            if (item < 16 * NOB * 18)
                wraw[u] = *reinterpret_cast<const cm_u32x4*>(P + ((size_t)(o0 + row) * 9 + rem / 2) * cols + cc + 8 * (rem & 1));
        }
    };
    load_chunk(0);
    load_weights(0);
    for (int cc = 0; cc < cols; cc += CM_CK) {
        __syncthreads();   // the previous chunk's fragments are read
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int item = tid + 256 * u;
            const int row = item / 18, rem = item - row * 18;
            if (item < 16 * NOB * 18)
                *reinterpret_cast<cm_u32x4*>(&wsm[row * CM_WSTR + (rem / 2) * CM_CK + 8 * (rem & 1)]) = wraw[u];
        }
#pragma unroll
        for (int u = 0; u < NIT; ++u) {
            if (s_lds[u] < 0) continue;
            unsigned part[PLANES][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                cm_f32x2 a = {raw[u][2 * q], raw[u][2 * q + 1]};
#pragma unroll
                for (int pl = 0; pl < PLANES; ++pl) {
                    const unsigned h = cm_bf16x2_bits(a);   // both rounded to nearest (even), packed
                    part[pl][q] = h;
                    if (pl + 1 < PLANES) {                 // exact: the remainders of a round to nearest
                        a.x -= __uint_as_float(h << 16);
                        a.y -= __uint_as_float(h & 0xFFFF0000u);
                    }
                }
            }
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl)
                *reinterpret_cast<uint4*>(&sbuf[pl * XS + s_lds[u]]) = make_uint4(part[pl][0], part[pl][1], part[pl][2], part[pl][3]);
        }
        __syncthreads();
        if (cc + CM_CK < cols) {   // the next chunk's input and weights, in flight during this chunk's products
            load_chunk(cc + CM_CK);
            load_weights(cc + CM_CK);
        }
#pragma unroll 1
        for (int st = 0; st < 5; ++st) {
            const int t = 2 * st + (g >> 1);                 // this lane group's tap (9: none)
            const int tt = t < 9 ? t : 8;
            const int dy = tt / 3, dx = tt - 3 * (tt / 3);
            cm_bf16x8 a[NOB];
#pragma unroll
            for (int ob = 0; ob < NOB; ++ob) {
                const cm_bf16x8 w8 = *reinterpret_cast<const cm_bf16x8*>(&wsm[(ob * 16 + l16) * CM_WSTR + tt * CM_CK + half]);
                a[ob] = t < 9 ? w8 : cm_bf16x8{};
            }
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) {
                const int so = ((wave + dy) * (CM_TC + 2) + pb * 16 + l16 + dx) * CM_PSTR + half;
#pragma unroll
                for (int pl = 0; pl < PLANES; ++pl) {
                    const cm_bf16x8 b = *reinterpret_cast<const cm_bf16x8*>(&sbuf[pl * XS + so]);
#pragma unroll
                    for (int ob = 0; ob < NOB; ++ob)
                        acc[ob][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ob], b, acc[ob][pb], 0, 0, 0);
                }
            }
        }
    }
    // epilogue: lane holds C[o = ob 16 + 4 g + j][pixel = pb 16 + l16] of tile
    // row `wave`; per 16-channel block it goes through the wave's staging rows
    // E[16][CM_EST] and out as 16-byte stores, 16 lanes per channel row of the
    // tile.  A wave's shared-memory accesses take effect in program order, so
    // the wave-scope fences between its writes and reads order the lanes.
    const int row = r0 + wave;
    __syncthreads();   // every wave's last fragment reads are done: the operand buffers become staging
    float* Eb = reinterpret_cast<float*>(sbuf) + wave * 16 * CM_EST;
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
        if (ob > 0) {   // the previous block's reads come first
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = o0 + ob * 16 + 4 * g + j;
            const float bo = (bias && o < co) ? bias[o] : 0.0f;
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) {
                float v = acc[ob][pb][j] + bo;
                if (relu && v < 0.0f) v = 0.0f;
                if (round_out) v = __uint_as_float(cm_bf16_bits(v) << 16);
                Eb[(4 * g + j) * CM_EST + pb * 16 + l16] = v;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (row < H) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ch = 4 * q + g, o = o0 + ob * 16 + ch, col = c0 + 4 * l16;
                if (o >= co) continue;
                const float4 v = *reinterpret_cast<const float4*>(&Eb[ch * CM_EST + 4 * l16]);
                float* dst = out + ((size_t)n * co + o) * npx + (size_t)row * W + col;
                if (col + 3 < W && (W & 3) == 0) {
                    *reinterpret_cast<float4*>(dst) = v;
                } else {
                    if (col < W) dst[0] = v.x;
                    if (col + 1 < W) dst[1] = v.y;
                    if (col + 2 < W) dst[2] = v.z;
                    if (col + 3 < W) dst[3] = v.w;
                }
            }
        }
    }
}

// Weight gradients of one 3 x 3 layer of the BF16 network on the matrix
// cores, per pixel chunk: dW[o][c][t] = sum_p g[o][p] in[c][p + off_t] and
// db[o] = sum_p g[o][p] (the chunks are added in order by k_wgrad_sum).  The
// layer input is BF16-valued (the BF16 network rounds every convolution
// input) and the output gradient g FP32, split into three BF16 parts
// (g = hi + mid + lo exactly), so every product is exact and the sums are
// FP32 in the matrix cores' order.  The contraction runs over pixels: one
// MFMA step (K = 32) takes 32 consecutive pixels of a row; lane l holds
// A[o = l % 16][8 (l / 16) + j] = g[o][pixel] and B[8 (l / 16) + j][c = l % 16]
// = in[c][pixel + off_t].  A chunk is WGM_ROWS rows x WGM_TC columns of one
// image, walked in sub-tiles of WGM_SR rows; each sub-tile's input (16
// channels, rows -1 .. WGM_SR, the tile's columns shifted by -1, 0 and +1:
// three copies, so that every tap's fragment is an aligned 16-byte read) is
// staged in shared memory as BF16, [copy][channel][row][column] with the
// channel stride padded by 8 BF16 so that the 16 lanes of a fragment read
// land on distinct banks.  Wave w takes output channels 16 w .. 16 w + 15.
// grid (N wgm_chunks(H, W), ceil(ci / 16)), block 256.  Writes
// part[chunk][o][c][t] for o < co, c < ci, and (input-channel block 0)
// bpart[chunk][o].  W must be a multiple of 8.
#define WGM_TC 64
#define WGM_SR 4
#define WGM_ROWS 16
#define WGM_CSTR ((WGM_SR + 2) * WGM_TC + 8)   // BF16 per staged channel

SMSM_HD inline int wgm_chunks(int H, int W) {
    return ((H + WGM_ROWS - 1) / WGM_ROWS) * ((W + WGM_TC - 1) / WGM_TC);
}

__global__ void __launch_bounds__(256, 2)
k_wgrad_mfma(int ci, int co, int H, int W, const float* __restrict__ in, const float* __restrict__ g,
             float* __restrict__ part, float* __restrict__ bpart) {
    __shared__ __attribute__((aligned(16))) unsigned short xs[3][16 * WGM_CSTR];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int gq = lane >> 4, l16 = lane & 15;
    const int cpi = wgm_chunks(H, W);
    const int chunk = blockIdx.x, n = chunk / cpi, cr = chunk - n * cpi;
    const int tiles_x = (W + WGM_TC - 1) / WGM_TC;
    const int ty = cr / tiles_x, tx = cr - ty * tiles_x;
    const int yc = ty * WGM_ROWS, x0 = tx * WGM_TC;
    const int c0 = blockIdx.y * 16;
    const size_t npx = (size_t)H * W;
    const float* src = in + (size_t)n * ci * npx;
    const int o = 16 * w + l16;                          // this lane's row of A
    const float* grow = g + ((size_t)n * co + (o < co ? o : 0)) * npx;
    cm_f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = cm_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    // output gradients of step s of the sub-tile at row y0 (8 pixels of this
    // lane's row o): loaded one step ahead of their products
    auto gload = [&](int y0, int s, cm_f32x4& u0, cm_f32x4& u1) __attribute__((always_inline)) {
        const int y = y0 + (s >> 1), xl = 32 * (s & 1) + 8 * gq;
        if (o < co && y < H && x0 + xl < W) {
            const cm_f32x4* gp = reinterpret_cast<const cm_f32x4*>(grow + (size_t)y * W + x0 + xl);
            u0 = gp[0];
            u1 = gp[1];
        } else {
            u0 = cm_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            u1 = u0;
        }
    };
    for (int sr = 0; sr < WGM_ROWS; sr += WGM_SR) {
        const int y0 = yc + sr;
        if (y0 >= H) break;                              // the same for the whole workgroup
        cm_f32x4 gn0, gn1;
        gload(y0, 0, gn0, gn1);                          // in flight during the staging
        __syncthreads();                                 // the previous sub-tile's fragments are read
        // items (channel, row, 8-column block), each written as three shifted copies
        for (int it = tid; it < 16 * (WGM_SR + 2) * (WGM_TC / 8); it += 256) {
            const int b = it % (WGM_TC / 8), rc = it / (WGM_TC / 8);
            const int r = rc % (WGM_SR + 2), c = rc / (WGM_SR + 2);
            const int y = y0 - 1 + r, cg = c0 + c, xb = x0 + 8 * b;
            const bool rok = cg < ci && y >= 0 && y < H;
            const float* row = src + (size_t)(rok ? cg : 0) * npx + (size_t)(rok ? y : 0) * W;
            float v[10];
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                const int x = xb - 1 + q;
                v[q] = (rok && x >= 0 && x < W) ? row[x] : 0.0f;
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {                // copy d holds in[..][x + d - 1]
                unsigned pk[4];   // the inputs are BF16 values: their upper halves, packed in pairs
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    pk[q] = __builtin_amdgcn_perm(__float_as_uint(v[2 * q + 1 + d]), __float_as_uint(v[2 * q + d]),
                                                  0x07060302u);
                *reinterpret_cast<uint4*>(&xs[d][c * WGM_CSTR + r * WGM_TC + 8 * b]) =
                    make_uint4(pk[0], pk[1], pk[2], pk[3]);
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int s = 0; s < 2 * WGM_SR; ++s) {
            const int ry = s >> 1, xl = 32 * (s & 1) + 8 * gq;   // this lane's 8 pixels: row y0 + ry, columns x0 + xl ..
            float gv[8];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                gv[q] = gn0[q];
                gv[4 + q] = gn1[q];
            }
            if (s + 1 < 2 * WGM_SR) gload(y0, s + 1, gn0, gn1);
#pragma unroll
            for (int q = 0; q < 8; ++q) bsum += gv[q];
            // g = hi + mid + lo, each part the upper half of what the previous
            // ones left (a truncation): every subtraction is exact and the
            // third remainder has at most 8 significant bits, so lo is exact.
            cm_bf16x8 a[3];
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                unsigned pk[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const unsigned b0 = __float_as_uint(gv[2 * q]), b1 = __float_as_uint(gv[2 * q + 1]);
                    pk[q] = __builtin_amdgcn_perm(b1, b0, 0x07060302u);
                    gv[2 * q] -= __uint_as_float(b0 & 0xFFFF0000u);
                    gv[2 * q + 1] -= __uint_as_float(b1 & 0xFFFF0000u);
                }
                a[pl] = __builtin_bit_cast(cm_bf16x8, make_uint4(pk[0], pk[1], pk[2], pk[3]));
            }
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3, dx = t - 3 * (t / 3);
                const cm_bf16x8 bfr =
                    *reinterpret_cast<const cm_bf16x8*>(&xs[dx][l16 * WGM_CSTR + (ry + dy) * WGM_TC + xl]);
#pragma unroll
                for (int pl = 0; pl < 3; ++pl)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[pl], bfr, acc[t], 0, 0, 0);
            }
        }
    }
    // lane holds C[o = 16 w + 4 gq + j][c = c0 + l16] of each tap
    const int c = c0 + l16;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int oo = 16 * w + 4 * gq + j;
        if (oo >= co || c >= ci) continue;
        float* dst = part + (((size_t)chunk * co + oo) * ci + c) * 9;
#pragma unroll
        for (int t = 0; t < 9; ++t) dst[t] = acc[t][j];
    }
    // bias: the four lane groups of a row add in a fixed order
    bsum += __shfl_xor(bsum, 16);
    bsum += __shfl_xor(bsum, 32);
    if (blockIdx.y == 0 && gq == 0 && o < co) bpart[(size_t)chunk * co + o] = bsum;
}

// x <- x rounded to a BF16 value (in place; the BF16 network's input).
__global__ void k_round_bf16(long n, float* __restrict__ x) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        x[k] = __uint_as_float(cm_bf16_bits(x[k]) << 16);
}
