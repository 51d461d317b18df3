// Warm-start network: six 3x3 "same" convolutions (3 -> 32 -> 32 -> 32 -> 32
// -> 32 -> 3, ReLU after the first five, biases) with the residual output
// X0 = C + f(C), trained on RTG-GMRES solutions with the mean squared error
// and Adam.  All kernels are bfloat16 MFMA (v_mfma_f32_16x16x32_bf16) with
// float32 accumulation; master weights and Adam moments are float32.
//
// Activations are NHWC bfloat16 with S in {8, 32} stored channels (the
// 3-channel tensors are padded with zeros to 8 = 16 bytes per pixel); the
// pixel index is i1 + I1 * i2 (i1 fastest, as in the solver's tensors).
// Weights are stored as W[co][k], k = tap * S_in + ci, tap = 3 t1 + t2 with
// t1, t2 the offsets + 1 along i1 and i2, rows padded to the MFMA tile (16 or
// 32) and k padded to a multiple of 32 with zeros.
//
// Convolution (implicit GEMM): D[co][pixel] = sum_k W[co][k] patch[k][pixel];
// the MFMA A operand is a weight row (from LDS), the B operand the lane's
// pixel with 8 consecutive k (one tap, 8 channels: one 16-byte load).
// Epilogues: bias + ReLU (hidden layers); X0 = C + out (inference);
// X0, squared error and the loss gradient (training); for the backward data
// pass the same kernel runs on flipped, transposed weights and masks the
// result with the ReLU of the layer input.
// Weight gradient: dW[co][tap, ci] = sum_pixels g[pixel][co] x[pixel + tap][ci]
// on MFMA with K = pixels (both operands staged transposed in LDS), per-
// workgroup partials reduced in a fixed order (deterministic).
#include "rtg_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace rtg {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

// two floats to bfloat16 (round to nearest even) in one 32-bit word, the
// first in the low half: one packed conversion instead of two
__device__ __forceinline__ unsigned bf2pack(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f2v{lo, hi}, bf2v));
}

enum ConvMode { CV_HIDDEN = 0, CV_LAST_INFER = 1, CV_LAST_TRAIN = 2, CV_BWD_DATA = 3 };

constexpr int kpad_of(int s) { return ((9 * s + 31) / 32) * 32; }

struct ConvArgs {
    int N, I1, I2;
    const bf16_t* x;      // NHWC input
    const bf16_t* w;      // [COUT_M][KPAD]
    const float* bias;    // [COUT_M] (hidden / last layers)
    bf16_t* out;          // NHWC output (activation or gradient)
    const bf16_t* mask;   // backward data: layer input whose positivity masks the result
    const float* C;       // last layer: observation, [N][3][I2][I1]
    const float* Y;       // training: target, [N][3][I2][I1]
    float* X0;            // inference: X0 = C + f(C), [N][3][I2][I1]
    float* loss_part;     // training: per-workgroup sum of squared errors
    float gscale;         // training: 2 / (number of target elements)
};

__device__ __forceinline__ bool bf_pos(bf16_t v) { return (v & 0x8000u) == 0 && (v & 0x7fffu) != 0; }

constexpr int CONV_TH = 8;               // output rows per tile (one wave per row)
constexpr int CONV_THREADS = 64 * CONV_TH;
constexpr int CONV_MAX_WG = 2 * 256;     // persistent grid: two workgroups per compute unit

// Tiles are 64 pixels along i1 by CONV_TH rows.  The grid is persistent: a
// workgroup walks the tiles t = blockIdx.x, blockIdx.x + gridDim.x, ... and
// loads the next tile's input (with its one-pixel halo) into registers while
// it computes the current tile from LDS.
template <int CIN_S, int COUT_M, int COUT_S, int MODE>
__global__ void __launch_bounds__(CONV_THREADS) k_conv(ConvArgs a) {
    constexpr int KPAD = kpad_of(CIN_S);
    constexpr int KQ = KPAD / 32;
    constexpr int KL = KPAD + 8;          // padded LDS row (bank spread), 16-byte multiple
    constexpr int MT = COUT_M / 16;
    constexpr int TW = 64, TH = CONV_TH;
    constexpr int NTH = CONV_THREADS;
    constexpr int HW = TW + 2, HH = TH + 2;
    constexpr int PS = CIN_S + 8;         // padded channels per staged pixel
    constexpr int NCH = CIN_S / 8;
    constexpr int NST = (HH * HW * NCH + NTH - 1) / NTH;
    constexpr bool LAST = MODE == CV_LAST_INFER || MODE == CV_LAST_TRAIN;
    __shared__ bf16_t Wl[COUT_M * KL];
    __shared__ bf16_t Xs[HH * HW * PS];
    __shared__ float red[CONV_TH];
    __shared__ float Bl[COUT_M];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n16 = lane & 15, s = lane >> 4;
    const int I1 = a.I1, I2 = a.I2;
    const size_t plane = (size_t)I1 * I2;
    const int nt1 = (I1 + TW - 1) / TW, nt2 = (I2 + TH - 1) / TH;
    const int ntiles = a.N * nt1 * nt2;
    for (int e = tid; e < COUT_M * (KPAD / 8); e += NTH) {
        const int row = e / (KPAD / 8), c8 = e % (KPAD / 8);
        *(u4*)(Wl + row * KL + c8 * 8) = *gptr((const u4*)(a.w + (size_t)row * KPAD + c8 * 8));
    }
    if (tid < COUT_M) Bl[tid] = (MODE == CV_BWD_DATA) ? 0.f : a.bias[tid];
    __syncthreads();
    // bias of the lane's four output rows per M tile (read from LDS, so that no
    // use inside the tile loop waits on global loads)
    float bias[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) bias[mt][i] = Bl[16 * mt + 4 * s + i];

    // input tile of tile t into registers (zero outside the image); loads are
    // unconditional from clamped addresses so that they all stay in flight
    u4 stg[NST];
    unsigned okbits = 0;
    auto fetch = [&](int t) {
        okbits = 0;
        const int t1 = t % nt1, r = t / nt1;
        const int i10 = t1 * TW, i20 = (r % nt2) * TH, img = r / nt2;
#pragma unroll
        for (int it = 0; it < NST; ++it) {
            const int e = tid + NTH * it;
            const int c8 = e % NCH, pxl = e / NCH;
            const int y1 = i10 - 1 + pxl % HW, y2 = i20 - 1 + pxl / HW;
            const int c1 = min(max(y1, 0), I1 - 1), c2 = min(max(y2, 0), I2 - 1);
            stg[it] = *gptr((const u4*)(a.x + (((size_t)img * I2 + c2) * I1 + c1) * CIN_S + c8 * 8));
            // the zero padding is applied when the registers go to LDS, so
            // that nothing waits for these loads before then
            okbits |= (unsigned)((e < HH * HW * NCH) & (y1 >= 0) & (y1 < I1) & (y2 >= 0) & (y2 < I2)) << it;
        }
    };
    float lsum = 0.f;
    int t = blockIdx.x;
    if (t < ntiles) fetch(t);
    for (; t < ntiles; t += gridDim.x) {
        const int t1 = t % nt1, r = t / nt1;
        const int i10 = t1 * TW, i2 = (r % nt2) * TH + wave, img = r / nt2;
        const bool row_ok = i2 < I2;
        const int i2c = min(i2, I2 - 1);
        __syncthreads();                  // the previous tile's reads of Xs are done
#pragma unroll
        for (int it = 0; it < NST; ++it) {
            const int e = tid + NTH * it;
            if (e < HH * HW * NCH) {
                const int c8 = e % NCH, pxl = e / NCH;
                const unsigned m = 0u - ((okbits >> it) & 1u);
                *(u4*)(Xs + pxl * PS + c8 * 8) = stg[it] & u4{m, m, m, m};
            }
        }
        __syncthreads();
        // epilogue operands of this tile, loaded before the next tile's input
        // so that waiting for them does not wait for the prefetch
        float cin[4][3], yin[4][3];
        u2 mk[4][MT];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int i1c = min(i10 + nt * 16 + n16, I1 - 1);
            if constexpr (LAST) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const size_t po = ((size_t)img * 3 + c) * plane + (size_t)i2c * I1 + i1c;
                    cin[nt][c] = *gptr(a.C + po);
                    if constexpr (MODE == CV_LAST_TRAIN) yin[nt][c] = *gptr(a.Y + po);
                }
            }
            if constexpr (MODE == CV_BWD_DATA) {
                const size_t pix = ((size_t)img * I2 + i2c) * I1 + i1c;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) mk[nt][mt] = *gptr((const u2*)(a.mask + pix * COUT_S + 16 * mt + 4 * s));
            }
        }
        __builtin_amdgcn_sched_barrier(0);   // keep those loads ahead of the prefetch
        fetch(min(t + (int)gridDim.x, ntiles - 1));   // the last tile loads a valid tile again, unused

        f4 acc[4][MT];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[nt][mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            bf8 A[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                A[mt] = __builtin_bit_cast(bf8, *(const u4*)(Wl + (16 * mt + n16) * KL + 32 * q + 8 * s));
            const int k = 32 * q + 8 * s;
            const int tap = k / CIN_S, ci0 = k % CIN_S;
            const int tp = tap < 9 ? tap : 0;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int il = nt * 16 + n16;
                const u4 v = *(const u4*)(Xs + ((wave + tp % 3) * HW + il + tp / 3) * PS + ci0);
                const bf8 B = __builtin_bit_cast(bf8, tap < 9 ? v : u4{0u, 0u, 0u, 0u});
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B, acc[nt][mt], 0, 0, 0);
            }
        }
        // values for every lane first (so that no load is sunk into the
        // guarded stores, where waiting for it would also wait for the
        // prefetch), then the guarded stores
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int i1 = i10 + nt * 16 + n16;
            const bool ok = row_ok && i1 < I1;
            const size_t pix = ((size_t)img * I2 + i2c) * I1 + min(i1, I1 - 1);
            if constexpr (MODE == CV_HIDDEN || MODE == CV_BWD_DATA) {
                u2 pk[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    float v[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        v[i] = acc[nt][mt][i];
                        if constexpr (MODE == CV_HIDDEN) v[i] = fmaxf(v[i] + bias[mt][i], 0.f);
                    }
                    if constexpr (MODE == CV_BWD_DATA) {
                        const u2 m2 = mk[nt][mt];
                        const bf16_t mb[4] = {(bf16_t)(m2[0] & 0xffffu), (bf16_t)(m2[0] >> 16),
                                              (bf16_t)(m2[1] & 0xffffu), (bf16_t)(m2[1] >> 16)};
#pragma unroll
                        for (int i = 0; i < 4; ++i) v[i] = bf_pos(mb[i]) ? v[i] : 0.f;
                    }
                    pk[mt][0] = (unsigned)f2bf(v[0]) | ((unsigned)f2bf(v[1]) << 16);
                    pk[mt][1] = (unsigned)f2bf(v[2]) | ((unsigned)f2bf(v[3]) << 16);
                }
                if (ok) {
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) *gptr_w((u2*)(a.out + pix * COUT_S + 16 * mt + 4 * s)) = pk[mt];
                }
            } else {
                // last layer: rows 0..2 of the first M tile (lanes with s = 0)
                // are the three output channels
                float x0[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) x0[c] = cin[nt][c] + acc[nt][0][c] + bias[0][c];
                const bool own = ok && s == 0;
                if constexpr (MODE == CV_LAST_INFER) {
                    if (own) {
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            *gptr_w(a.X0 + ((size_t)img * 3 + c) * plane + (size_t)i2 * I1 + i1) = x0[c];
                    }
                } else {
                    bf16_t gb[8];
                    float l = 0.f;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float dlt = x0[c] - yin[nt][c];
                        l += dlt * dlt;
                        gb[c] = f2bf(a.gscale * dlt);
                    }
#pragma unroll
                    for (int c = 3; c < 8; ++c) gb[c] = 0;
                    u4 pk;
#pragma unroll
                    for (int q = 0; q < 4; ++q) pk[q] = (unsigned)gb[2 * q] | ((unsigned)gb[2 * q + 1] << 16);
                    lsum += own ? l : 0.f;
                    if (own) *gptr_w((u4*)(a.out + pix * 8)) = pk;
                }
            }
        }
    }
    if constexpr (MODE == CV_LAST_TRAIN) {
        lsum = wave_sum(lsum);
        if (lane == 0) red[wave] = lsum;
        __syncthreads();
        if (tid == 0) {
            float tot = 0.f;
            for (int w = 0; w < CONV_TH; ++w) tot += red[w];
            a.loss_part[blockIdx.x] = tot;
        }
    }
}

struct WgradArgs {
    int N, I1, I2, rows;  // rows (i2) per workgroup
    const bf16_t* g;      // NHWC gradient at the layer output (COUT_S channels)
    const bf16_t* x;      // NHWC layer input (CIN_S channels)
    float* part;          // [workgroups][COUT_M * KPAD + COUT_M]
};

// ---------------------------------------------------------------------------
// Two consecutive 3x3 layers in one pass (inference).  Layer A (CIN -> 32,
// bias, ReLU) is evaluated on the output tile grown by one pixel on every
// side and kept in LDS as bfloat16 -- zero outside the image, which is the
// zero padding layer B sees -- and layer B (32 -> COUT) reads it from LDS, so
// the activation between the two layers never goes to memory.  Layer A's
// weights stay in registers for the whole kernel, layer B's in LDS.
// Both layers of a hidden pair run on v_mfma_f32_32x32x16_bf16 (32 output
// channels x 32 pixels per product): each 16-byte activation fragment read
// from LDS feeds twice the products of a 16x16x32 tile, which halves the
// LDS reads per product -- the bound of this kernel.  The last pair's
// layer B (3 output channels) keeps 16x16x32 tiles.
// Persistent grid: a workgroup streams the next tile's input (with its
// two-pixel halo) into LDS by asynchronous loads while it computes layer B of
// the current tile.
// ---------------------------------------------------------------------------
struct Conv2Args {
    int N, I1, I2;
    const bf16_t* x;       // NHWC input, CIN_S channels
    const bf16_t* wA;      // [32][KPAD(CIN_S)]
    const float* bA;       // [32]
    const bf16_t* wB;      // [COUTB_M][KPAD(32)]
    const float* bB;       // [COUTB_M]
    bf16_t* out;           // NHWC output, COUTB_S channels (hidden pair)
    const float* C;        // last pair: observation, [N][3][I2][I1]
    float* X0;             // last pair: X0 = C + f(C)
};

constexpr int C2_TH = 8, C2_TW = 64;
constexpr int C2_THREADS = 64 * C2_TH;
constexpr int C2_MAX_WG = 256;           // one workgroup per compute unit (LDS)

template <int CIN_S, int COUTB_M, int COUTB_S, bool LASTB>
__global__ void __launch_bounds__(C2_THREADS) k_conv2(Conv2Args a) {
    constexpr int TH = C2_TH, TW = C2_TW, NTH = C2_THREADS;
    constexpr int IH = TH + 4, IW = TW + 4;            // input tile (two-pixel halo)
    constexpr int MH = TH + 2, MW = TW + 2;            // layer-A tile (one-pixel halo)
    constexpr int MP = MH * MW;                         // layer-A pixels
    constexpr int MNT = (MP + 31) / 32;                 // layer-A N-tiles of 32 pixels
    constexpr int KSA = (9 * CIN_S + 15) / 16;          // layer-A K steps of 16 (taps x channels)
    constexpr int DA = KSA % 3 == 0 ? 3 : KSA;          // layer-A operand reads ahead
    constexpr int PSA = CIN_S + 8, PSB = 32 + 8;        // padded channels per pixel in LDS
    constexpr int KPA = kpad_of(CIN_S), KQA = KPA / 32;
    constexpr int KPB = kpad_of(32), KQB = KPB / 32;
    constexpr int MTB = COUTB_M / 16;
    constexpr int NCH = CIN_S / 8;
    constexpr int KLB = KPB + 8;                        // padded LDS row of layer-B weights
    __shared__ __attribute__((aligned(16))) bf16_t Xs[IH * IW * PSA];
    __shared__ __attribute__((aligned(16))) bf16_t Ms[MNT * 32 * PSB];   // whole N-tiles: unconditional stores
    __shared__ __attribute__((aligned(16))) bf16_t WlB[COUTB_M * KLB];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: a scalar N-tile loop
    const int n16 = lane & 15, s = lane >> 4;
    const int n32 = lane & 31, g = lane >> 5;
    const int I1 = a.I1, I2 = a.I2;
    const size_t plane = (size_t)I1 * I2;
    const int nt1 = (I1 + TW - 1) / TW, nt2 = (I2 + TH - 1) / TH;
    const int ntiles = a.N * nt1 * nt2;

    // layer-A weights (MFMA A operands of 32x32x16 products, reused by every
    // N-tile) in registers; layer-B weights in LDS; biases in registers (the
    // lane's 16 output channels of a 32x32 result: 8 (v / 4) + 4 g + v % 4)
    bf8 AfA[KSA];
#pragma unroll
    for (int q = 0; q < KSA; ++q)
        AfA[q] = __builtin_bit_cast(bf8, *gptr((const u4*)(a.wA + (size_t)n32 * KPA + 16 * q + 8 * g)));
    for (int e = tid; e < COUTB_M * (KPB / 8); e += NTH) {
        const int row = e / (KPB / 8), c8 = e % (KPB / 8);
        *(u4*)(WlB + row * KLB + c8 * 8) = *gptr((const u4*)(a.wB + (size_t)row * KPB + c8 * 8));
    }
    f16v biasA, biasB = {};                             // 32x32 results (hidden layers)
    float biasL[4 * MTB];                               // last pair's layer B (16x16 results)
#pragma unroll
    for (int v = 0; v < 16; ++v) biasA[v] = *gptr(a.bA + 8 * (v / 4) + 4 * g + v % 4);
    if constexpr (LASTB) {
#pragma unroll
        for (int mt = 0; mt < MTB; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) biasL[4 * mt + i] = *gptr(a.bB + 16 * mt + 4 * s + i);
    } else {
#pragma unroll
        for (int v = 0; v < 16; ++v) biasB[v] = *gptr(a.bB + 8 * (v / 4) + 4 * g + v % 4);
    }

    // The input tile (two-pixel halo) reaches Xs by asynchronous global-to-
    // LDS loads: 16-byte slots, PSA / 8 per pixel, slot s fetched by thread
    // s % NTH of pass s / NTH (a wave's instruction fills 1 KB, lane i at
    // bytes 16 i).  Padding slots and pixels outside the image are fetched
    // from past the buffer range and read as zeros.  The next tile's loads
    // are issued once layer A no longer reads Xs, one pass every other step
    // of layer B's products.
    constexpr int SPP = PSA / 8;                        // slots per pixel
    constexpr int NSL = IH * IW * SPP;
    constexpr int NPASS = (NSL + NTH - 1) / NTH;        // passes; the last one may be partial
    const auto rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16_t*>(a.x), (short)0,
                                                      (int)((size_t)a.N * plane * CIN_S * 2), 0x00020000);
    const auto ro = __builtin_amdgcn_make_buffer_rsrc(a.out, (short)0, (int)((size_t)a.N * plane * COUTB_S * 2),
                                                      0x00020000);
    constexpr int NSTB = 8;                             // hidden pair: stores per wave and tile
    static_assert(NSTB < 16, "vmcnt field");
    struct Origin { int i10, i20, img; };
    auto origin = [&](int tt) {
        const int t1 = tt % nt1, r = tt / nt1;
        return Origin{t1 * TW, (r % nt2) * TH, r / nt2};
    };
    auto dma_pass = [&](const Origin& o, int it) {
        const int sl = it * NTH + tid;
        if (NSL % NTH != 0 && it == NPASS - 1 && sl >= NSL) return;
        const int pxl = sl / SPP, c = sl % SPP;
        const int y1 = o.i10 - 2 + pxl % IW, y2 = o.i20 - 2 + pxl / IW;
        const bool ok = (c < NCH) & (y1 >= 0) & (y1 < I1) & (y2 >= 0) & (y2 < I2);
        const unsigned off =
            ok ? (unsigned)(((((size_t)o.img * I2 + y2) * I1 + y1) * CIN_S + c * 8) * 2) : 0x80000000u;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rx, (__attribute__((address_space(3))) void*)(Xs + (size_t)(it * NTH + wave * 64) * 8), 16, off, 0, 0, 0);
    };
    int t = blockIdx.x;
    if (t < ntiles) {
        const Origin o0 = origin(t);
#pragma unroll
        for (int it = 0; it < NPASS; ++it) dma_pass(o0, it);
    }
    for (; t < ntiles; t += gridDim.x) {
        const int t1 = t % nt1, rr = t / nt1;
        const int i10 = t1 * TW, i20 = (rr % nt2) * TH, img = rr / nt2;
        // this wave's loads of the tile have landed: memory operations
        // complete in issue order, and after the input loads a hidden pair's
        // wave has issued exactly NSTB stores, which need not be waited for
        if (LASTB || t == (int)blockIdx.x) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        else __builtin_amdgcn_s_waitcnt(0x0F70 | NSTB);                         // vmcnt(NSTB)
        __syncthreads();                     // all of them; the previous tile's reads of Ms are done
        // epilogue operands of layer B (last pair)
        float cin[4][3];
        const int i2 = i20 + wave;
        const int i2c = min(i2, I2 - 1);
        if constexpr (LASTB) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int i1c = min(i10 + nt * 16 + n16, I1 - 1);
#pragma unroll
                for (int c = 0; c < 3; ++c) cin[nt][c] = *gptr(a.C + ((size_t)img * 3 + c) * plane + (size_t)i2c * I1 + i1c);
            }
        }


        // ---- layer A on the grown tile: N-tiles of 32 pixels (32x32x16
        // products: lane l holds pixel nt 32 + l % 32 and, of each K step of
        // 16, the 8 channels 8 (l / 32) ..), wave w takes w, w + 8, ...
        // Operand reads run DA steps ahead of the matrix cores, across the
        // end of an N-tile into the wave's next one (DA divides KSA, so step
        // q always sits in slot q % DA).
        static_assert(KSA % DA == 0, "operand window");
        auto readA = [&](int nt, int q) {
            const int pc = min(nt * 32 + n32, MP - 1);
            const int mr = pc / MW, mc = pc % MW;
            const int k = 16 * q + 8 * g;
            const int tap = k / CIN_S, ci0 = k % CIN_S;
            const int tp = tap < 9 ? tap : 0;
            const u4 v = *(const u4*)(Xs + ((mr + tp % 3) * IW + mc + tp / 3) * PSA + ci0);
            return tap < 9 ? v : u4{0u, 0u, 0u, 0u};
        };
        {
            u4 Bw[DA];
#pragma unroll
            for (int q = 0; q < DA; ++q) Bw[q] = readA(min(wave, MNT - 1), q);
            for (int nt = wave; nt < MNT; nt += TH) {
                const int ntn = min(nt + TH, MNT - 1);          // past the last tile: a valid tile again, unused
                f16v acc = biasA;                           // the bias enters as the first accumulator
#pragma unroll
                for (int q = 0; q < KSA; ++q) {
                    const u4 cur = Bw[q % DA];
                    Bw[q % DA] = (q + DA < KSA) ? readA(nt, q + DA) : readA(ntn, q + DA - KSA);
                    __builtin_amdgcn_sched_barrier(0);       // keep the read ahead of this product
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AfA[q], __builtin_bit_cast(bf8, cur), acc, 0, 0, 0);
                }
                // epilogue without branches: ReLU as a clamp to [0, lim], with
                // lim = 0 for pixels outside the image (the zero padding of
                // layer B's input); the pixels past MP of the last N-tile land
                // in Ms's tail
                const int p = nt * 32 + n32;
                const int pc = min(p, MP - 1);
                const int mr = pc / MW, mc = pc % MW;
                const int y2 = i20 - 1 + mr, y1 = i10 - 1 + mc;
                const float lim = ((y1 >= 0) & (y1 < I1) & (y2 >= 0) & (y2 < I2)) ? __builtin_inff() : 0.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    u2 pk;
                    pk[0] = bf2pack(__builtin_amdgcn_fmed3f(acc[4 * r], 0.f, lim),
                                    __builtin_amdgcn_fmed3f(acc[4 * r + 1], 0.f, lim));
                    pk[1] = bf2pack(__builtin_amdgcn_fmed3f(acc[4 * r + 2], 0.f, lim),
                                    __builtin_amdgcn_fmed3f(acc[4 * r + 3], 0.f, lim));
                    *(u2*)(Ms + p * PSB + 8 * r + 4 * g) = pk;
                }
            }
        }
        __syncthreads();                     // layer A done: Ms complete, Xs free
        const bool nxt = t + (int)gridDim.x < ntiles;
        const Origin on = origin(min(t + (int)gridDim.x, ntiles - 1));
        if constexpr (!LASTB) {
            // ---- layer B (hidden pair): wave w takes output row w, two
            // N-tiles of 32 pixels, 32x32x16 products; the operands (weights
            // and activations) of step q + 2 are read while step q is on the
            // matrix cores
            auto loadB2 = [&](int q, u4* Bq, u4& Wq) {
                const int k = 16 * q + 8 * g;
                const int tap = k / 32, ci0 = k % 32;
                Wq = *(const u4*)(WlB + n32 * KLB + k);
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    Bq[nt] = *(const u4*)(Ms + ((wave + tap % 3) * MW + nt * 32 + n32 + tap / 3) * PSB + ci0);
            };
            constexpr int KSB = 9 * 32 / 16;
            static_assert(2 * NPASS <= KSB + 1, "input passes per layer-B step");
            constexpr int PD = 2;                       // operand reads run PD steps ahead
            u4 Bb[PD + 1][2], Wb[PD + 1];
#pragma unroll
            for (int q = 0; q < PD; ++q) loadB2(q, Bb[q], Wb[q]);
            f16v accB[2] = {biasB, biasB};              // the bias enters as the first accumulator
#pragma unroll
            for (int q = 0; q < KSB; ++q) {
                if (q + PD < KSB) loadB2(q + PD, Bb[(q + PD) % (PD + 1)], Wb[(q + PD) % (PD + 1)]);
                if ((q & 1) == 0 && q / 2 < NPASS && nxt) dma_pass(on, q / 2);
                __builtin_amdgcn_sched_barrier(0);       // keep the reads ahead of these products
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    accB[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, Wb[q % (PD + 1)]),
                                                                       __builtin_bit_cast(bf8, Bb[q % (PD + 1)][nt]),
                                                                       accB[nt], 0, 0, 0);
            }
            const bool row_ok = i2 < I2;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int i1 = i10 + nt * 32 + n32;
                const bool ok = row_ok && i1 < I1;
                // buffer stores, issued by every lane (past the range for
                // pixels outside the image, which the hardware drops): each
                // wave issues exactly NSTB stores per tile after its input loads
                const unsigned off = ok ? (unsigned)(((((size_t)img * I2 + i2) * I1 + i1) * COUTB_S + 4 * g) * 2)
                                        : 0x80000000u;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    u2 pk;
                    pk[0] = bf2pack(fmaxf(accB[nt][4 * r], 0.f), fmaxf(accB[nt][4 * r + 1], 0.f));
                    pk[1] = bf2pack(fmaxf(accB[nt][4 * r + 2], 0.f), fmaxf(accB[nt][4 * r + 3], 0.f));
                    __builtin_amdgcn_raw_buffer_store_b64(pk, ro, off + 16u * r, 0, 0);
                }
            }
        } else {
            // ---- layer B: wave w takes output row w, four N-tiles of 16 pixels;
            // the operands (weights and activations) of tap q + 2 are read while
            // tap q is on the matrix cores
            f4 acc[4][MTB];
    #pragma unroll
            for (int nt = 0; nt < 4; ++nt)
    #pragma unroll
                for (int mt = 0; mt < MTB; ++mt) acc[nt][mt] = f4{0.f, 0.f, 0.f, 0.f};
            auto loadB = [&](int q, u4* Bq, u4* Wq) {
                const int k = 32 * q + 8 * s;
                const int tap = k / 32, ci0 = k % 32;
                const int tp = tap < 9 ? tap : 0;
    #pragma unroll
                for (int mt = 0; mt < MTB; ++mt) Wq[mt] = *(const u4*)(WlB + (16 * mt + n16) * KLB + 32 * q + 8 * s);
    #pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int il = nt * 16 + n16;
                    const u4 v = *(const u4*)(Ms + ((wave + tp % 3) * MW + il + tp / 3) * PSB + ci0);
                    Bq[nt] = tap < 9 ? v : u4{0u, 0u, 0u, 0u};
                }
            };
            {
                constexpr int PD = 2;                   // operand reads run PD taps ahead
                u4 Bb[PD + 1][4], Wb[PD + 1][MTB];
    #pragma unroll
                for (int q = 0; q < PD; ++q) loadB(q, Bb[q], Wb[q]);
    #pragma unroll
                for (int q = 0; q < KQB; ++q) {
                    if (q + PD < KQB) loadB(q + PD, Bb[(q + PD) % (PD + 1)], Wb[(q + PD) % (PD + 1)]);
                    static_assert(NPASS <= KQB, "input passes per layer-B tap");
                    if (q < NPASS && nxt) dma_pass(on, q);
                    __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of these products
    #pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
    #pragma unroll
                        for (int mt = 0; mt < MTB; ++mt)
                            acc[nt][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf8, Wb[q % (PD + 1)][mt]), __builtin_bit_cast(bf8, Bb[q % (PD + 1)][nt]),
                                acc[nt][mt], 0, 0, 0);
                }
            }
            const bool row_ok = i2 < I2;
    #pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int i1 = i10 + nt * 16 + n16;
                const bool ok = row_ok && i1 < I1;
                if constexpr (!LASTB) {
                    const size_t pix = ((size_t)img * I2 + i2c) * I1 + min(i1, I1 - 1);
                    u2 pk[MTB];
    #pragma unroll
                    for (int mt = 0; mt < MTB; ++mt) {
                        float v[4];
    #pragma unroll
                        for (int i = 0; i < 4; ++i) v[i] = fmaxf(acc[nt][mt][i] + biasL[4 * mt + i], 0.f);
                        pk[mt][0] = (unsigned)f2bf(v[0]) | ((unsigned)f2bf(v[1]) << 16);
                        pk[mt][1] = (unsigned)f2bf(v[2]) | ((unsigned)f2bf(v[3]) << 16);
                    }
                    if (ok) {
    #pragma unroll
                        for (int mt = 0; mt < MTB; ++mt) *gptr_w((u2*)(a.out + pix * COUTB_S + 16 * mt + 4 * s)) = pk[mt];
                    }
                } else {
                    // rows 0..2 of the first M tile (lanes with s = 0) are the three output channels
                    float x0[3];
    #pragma unroll
                    for (int c = 0; c < 3; ++c) x0[c] = cin[nt][c] + acc[nt][0][c] + biasL[c];
                    if (ok && s == 0) {
    #pragma unroll
                        for (int c = 0; c < 3; ++c) *gptr_w(a.X0 + ((size_t)img * 3 + c) * plane + (size_t)i2 * I1 + i1) = x0[c];
                    }
                }
            }
        }
    }
}

template <int CIN_S, int COUT_S, int COUT_M>
__global__ void __launch_bounds__(256) k_wgrad(WgradArgs a) {
    constexpr int KPAD = kpad_of(CIN_S);
    constexpr int TAPS = KPAD / CIN_S;    // 9, or 12 with zero padding
    constexpr int NT = KPAD / 16, MT = COUT_M / 16;
    constexpr int TILES = NT * MT;
    constexpr int SLOTS = (TILES + 3) / 4;
    constexpr int PX = 32, PXL = PX + 8;  // pixels per chunk, padded LDS row
    __shared__ bf16_t gT[COUT_M * PXL];
    __shared__ bf16_t xs[TAPS * CIN_S * PXL];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n16 = lane & 15, s = lane >> 4;
    const int I1 = a.I1, I2 = a.I2;
    const int ngrp = (I2 + a.rows - 1) / a.rows;
    const int img = blockIdx.x / ngrp;
    const int r0 = (blockIdx.x % ngrp) * a.rows;

    for (int e = tid; e < COUT_M * PXL; e += 256) gT[e] = 0;
    f4 acc[SLOTS];
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) acc[u] = f4{0.f, 0.f, 0.f, 0.f};
    float dbacc = 0.f;

    for (int i2 = r0; i2 < min(r0 + a.rows, I2); ++i2) {
        for (int c0 = 0; c0 < I1; c0 += PX) {
            __syncthreads();
            // stage g^T: rows co < COUT_S (rows beyond stay zero)
            for (int e = tid; e < PX * (COUT_S / 8); e += 256) {
                const int px = e % PX, c8 = e / PX;
                const int i1 = c0 + px;
                const bool ok = i1 < I1;
                const u4 v = *gptr((const u4*)(a.g + (((size_t)img * I2 + i2) * I1 + min(i1, I1 - 1)) * COUT_S + c8 * 8));
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    gT[(c8 * 8 + 2 * t) * PXL + px] = ok ? (bf16_t)(v[t] & 0xffffu) : (bf16_t)0;
                    gT[(c8 * 8 + 2 * t + 1) * PXL + px] = ok ? (bf16_t)(v[t] >> 16) : (bf16_t)0;
                }
            }
            // stage the shifted input for every tap: xs[tap][ci][px] = x[i1 + t1 - 1, i2 + t2 - 1][ci]
            for (int e = tid; e < TAPS * PX * (CIN_S / 8); e += 256) {
                const int px = e % PX;
                const int r = e / PX;
                const int c8 = r % (CIN_S / 8), tap = r / (CIN_S / 8);
                const int y1 = c0 + px + tap / 3 - 1, y2 = i2 + tap % 3 - 1;
                const bool ok = tap < 9 && c0 + px < I1 && y1 >= 0 && y1 < I1 && y2 >= 0 && y2 < I2;
                const int c1 = min(max(y1, 0), I1 - 1), c2 = min(max(y2, 0), I2 - 1);
                const u4 v = *gptr((const u4*)(a.x + (((size_t)img * I2 + c2) * I1 + c1) * CIN_S + c8 * 8));
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    xs[(tap * CIN_S + c8 * 8 + 2 * t) * PXL + px] = ok ? (bf16_t)(v[t] & 0xffffu) : (bf16_t)0;
                    xs[(tap * CIN_S + c8 * 8 + 2 * t + 1) * PXL + px] = ok ? (bf16_t)(v[t] >> 16) : (bf16_t)0;
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < SLOTS; ++u) {
                const int t = wave + 4 * u;
                if (t < TILES) {
                    const int mt = t / NT, nt = t % NT;
                    const bf8 A = __builtin_bit_cast(bf8, *(const u4*)(gT + (16 * mt + n16) * PXL + 8 * s));
                    const bf8 B = __builtin_bit_cast(bf8, *(const u4*)(xs + (16 * nt + n16) * PXL + 8 * s));
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[u], 0, 0, 0);
                }
            }
            if (tid < COUT_M) {
                for (int px = 0; px < PX; ++px) dbacc += bf2f(gT[tid * PXL + px]);
            }
        }
    }
    float* part = a.part + (size_t)blockIdx.x * (COUT_M * KPAD + COUT_M);
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
        const int t = wave + 4 * u;
        if (t < TILES) {
            const int mt = t / NT, nt = t % NT;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                *gptr_w(part + (size_t)(16 * mt + 4 * s + i) * KPAD + 16 * nt + n16) = acc[u][i];
        }
    }
    if (tid < COUT_M) *gptr_w(part + COUT_M * KPAD + tid) = dbacc;
}

// out[e] = sum over parts in a fixed order (deterministic)
__global__ void k_reduce_parts(const float* __restrict__ part, int nparts, int len, float* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int w = 0;
    for (; w + 8 <= nparts; w += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += *gptr(part + (size_t)(w + u) * len + e);
    }
    for (; w < nparts; ++w) acc[0] += *gptr(part + (size_t)w * len + e);
    out[e] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// planar float32 [N][3][I2][I1] -> NHWC bfloat16 with 8 stored channels
__global__ void k_pack(const float* __restrict__ X, int N, int I1, int I2, bf16_t* __restrict__ out) {
    const size_t plane = (size_t)I1 * I2;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (size_t)N * plane) return;
    const size_t img = p / plane, r = p % plane;
    bf16_t v[8];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = f2bf(*gptr(X + (img * 3 + c) * plane + r));
#pragma unroll
    for (int c = 3; c < 8; ++c) v[c] = 0;
    u4 pk;
#pragma unroll
    for (int q = 0; q < 4; ++q) pk[q] = (unsigned)v[2 * q] | ((unsigned)v[2 * q + 1] << 16);
    *gptr_w((u4*)(out + p * 8)) = pk;
}

// Adam on a float32 array (bias-corrected; c1 = 1 - b1^t, c2 = 1 - b2^t)
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

// bfloat16 working copies of a layer: W (as stored) and the flipped,
// transposed weights of the backward data pass,
// Wt[ci][tap' * S_out + co] = W[co][(8 - tap') * S_in + ci].
__global__ void k_make_weights(const float* __restrict__ W, int cout_m, int kpad, int s_in,
                               bf16_t* __restrict__ Wh, bf16_t* __restrict__ Wt, int s_out, int kpad_t) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < cout_m * kpad) Wh[e] = f2bf(W[e]);
    if (Wt != nullptr && e < 32 * kpad_t) {
        const int ci = e / kpad_t, k = e % kpad_t;
        const int tapp = k / s_out, co = k % s_out;
        float v = 0.f;
        if (tapp < 9 && co < cout_m && ci < s_in) v = W[(size_t)co * kpad + (8 - tapp) * s_in + ci];
        Wt[e] = f2bf(v);
    }
}

}  // namespace rtg

// ---------------------------------------------------------------------------
// host side: network state, workspace and the C ABI
// ---------------------------------------------------------------------------
namespace {
using namespace rtg;

struct LayerDef {
    int cin, cout, s_in, s_out, cout_m;
};
constexpr int NL = 6;
const LayerDef LAYERS[NL] = {
    {3, 32, 8, 32, 32}, {32, 32, 32, 32, 32}, {32, 32, 32, 32, 32},
    {32, 32, 32, 32, 32}, {32, 32, 32, 32, 32}, {32, 3, 32, 8, 16}};

size_t al(size_t x) { return (x + 255) / 256 * 256; }

struct LayerOff {
    size_t W, b, mW, vW, mb, vb, gW, gb, Wh, Wt;
    int kpad, kpad_t, nw, nb;
};

struct StateLayout {
    LayerOff L[NL];
    size_t total;
};

StateLayout state_layout() {
    StateLayout S{};
    size_t off = 0;
    auto take = [&](size_t bytes) { off = al(off); size_t at = off; off += bytes; return at; };
    for (int l = 0; l < NL; ++l) {
        const LayerDef& d = LAYERS[l];
        LayerOff& o = S.L[l];
        o.kpad = kpad_of(d.s_in);
        o.kpad_t = kpad_of(d.s_out);
        o.nw = d.cout_m * o.kpad;
        o.nb = d.cout_m;
        o.W = take(o.nw * 4);
        o.b = take(o.nb * 4);
        o.mW = take(o.nw * 4);
        o.vW = take(o.nw * 4);
        o.mb = take(o.nb * 4);
        o.vb = take(o.nb * 4);
        o.gW = take((o.nw + o.nb) * 4);        // gradient of W followed by that of b
        o.gb = o.gW + (size_t)o.nw * 4;
        o.Wh = take(o.nw * 2);
        o.Wt = take((size_t)32 * o.kpad_t * 2);
    }
    S.total = al(off);
    return S;
}

constexpr int WG_ROWS = 8;

struct WsLayout {
    size_t xin, act[NL - 1], g8, gA, gB, part, loss, total;
    int nconv, nwg;
};

WsLayout ws_layout(int N, int I1, int I2) {
    WsLayout W{};
    const size_t px = (size_t)N * I1 * I2;
    size_t off = 0;
    auto take = [&](size_t bytes) { off = al(off); size_t at = off; off += bytes; return at; };
    W.xin = take(px * 8 * 2);
    for (int l = 0; l < NL - 1; ++l) W.act[l] = take(px * 32 * 2);
    W.g8 = take(px * 8 * 2);
    W.gA = take(px * 32 * 2);
    W.gB = take(px * 32 * 2);
    W.nconv = std::min(N * ((I2 + CONV_TH - 1) / CONV_TH) * ((I1 + 63) / 64), CONV_MAX_WG);
    W.nwg = N * ((I2 + WG_ROWS - 1) / WG_ROWS);
    W.part = take((size_t)W.nwg * (32 * kpad_of(32) + 32) * 4);
    W.loss = take((size_t)W.nconv * 4 + 4);
    W.total = al(off);
    return W;
}

template <int CIN_S, int COUT_M, int COUT_S, int MODE>
hipError_t conv(const ConvArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_conv<CIN_S, COUT_M, COUT_S, MODE>), dim3(grid), dim3(CONV_THREADS), 0, s, a);
    return hipGetLastError();
}

template <int CIN_S, int COUTB_M, int COUTB_S, bool LASTB>
hipError_t conv2(const Conv2Args& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_conv2<CIN_S, COUTB_M, COUTB_S, LASTB>), dim3(grid), dim3(C2_THREADS), 0, s, a);
    return hipGetLastError();
}

template <int CIN_S, int COUT_S, int COUT_M>
hipError_t wgrad(const WgradArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_wgrad<CIN_S, COUT_S, COUT_M>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

// forward of layer l (0-based) into out / X0
hipError_t layer_forward(int l, char* st, const StateLayout& S, const bf16_t* x, bf16_t* out, const float* C,
                         const float* Y, float* X0, float* loss_part, float gscale, int N, int I1, int I2,
                         int grid, bool train, hipStream_t s) {
    const LayerOff& o = S.L[l];
    ConvArgs a{};
    a.N = N; a.I1 = I1; a.I2 = I2;
    a.x = x;
    a.w = (const bf16_t*)(st + o.Wh);
    a.bias = (const float*)(st + o.b);
    a.out = out;
    a.C = C; a.Y = Y; a.X0 = X0; a.loss_part = loss_part; a.gscale = gscale;
    if (l == 0) return conv<8, 32, 32, CV_HIDDEN>(a, grid, s);
    if (l < NL - 1) return conv<32, 32, 32, CV_HIDDEN>(a, grid, s);
    if (train) return conv<32, 16, 8, CV_LAST_TRAIN>(a, grid, s);
    return conv<32, 16, 8, CV_LAST_INFER>(a, grid, s);
}

int check_dims(int N, int I1, int I2) {
    if (N < 1 || I1 < 1 || I2 < 1) return RTG_E_SHAPE;
    // the fused pairs address a 32-channel activation with 32-bit byte offsets
    if ((size_t)N * I1 * I2 * 32 * 2 > 0x7FFFFFFFull) return RTG_E_SHAPE;
    return RTG_OK;
}

}  // namespace

extern "C" {

size_t rtg_cnn_state_bytes(void) { return state_layout().total; }

size_t rtg_cnn_workspace_bytes(int N, int I1, int I2) {
    if (check_dims(N, I1, I2)) return 0;
    return ws_layout(N, I1, I2).total;
}

int rtg_cnn_init(void* state, const float* params, void* stream) {
    if (!state || !params) return RTG_E_ARG;
    const StateLayout S = state_layout();
    std::vector<unsigned char> host(S.total, 0);
    size_t pi = 0;
    for (int l = 0; l < NL; ++l) {
        const LayerDef& d = LAYERS[l];
        const LayerOff& o = S.L[l];
        float* W = (float*)(host.data() + o.W);
        float* b = (float*)(host.data() + o.b);
        for (int co = 0; co < d.cout; ++co)
            for (int t1 = 0; t1 < 3; ++t1)
                for (int t2 = 0; t2 < 3; ++t2)
                    for (int ci = 0; ci < d.cin; ++ci)
                        W[(size_t)co * o.kpad + (t1 * 3 + t2) * d.s_in + ci] = params[pi++];
        for (int co = 0; co < d.cout; ++co) b[co] = params[pi++];
    }
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(state, host.data(), S.total, hipMemcpyHostToDevice, s) != hipSuccess) return RTG_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RTG_E_HIP;
    for (int l = 0; l < NL; ++l) {
        const LayerDef& d = LAYERS[l];
        const LayerOff& o = S.L[l];
        char* st = (char*)state;
        const int n = std::max(o.nw, 32 * o.kpad_t);
        hipLaunchKernelGGL(k_make_weights, dim3((n + 255) / 256), dim3(256), 0, s, (const float*)(st + o.W),
                           d.cout_m, o.kpad, d.s_in, (bf16_t*)(st + o.Wh), l > 0 ? (bf16_t*)(st + o.Wt) : nullptr,
                           d.s_out, o.kpad_t);
    }
    return hipGetLastError() == hipSuccess ? RTG_OK : RTG_E_HIP;
}

static int export_arrays(const void* state, float* out, bool grads) {
    const StateLayout S = state_layout();
    std::vector<unsigned char> host(S.total);
    if (hipMemcpy(host.data(), state, S.total, hipMemcpyDeviceToHost) != hipSuccess) return RTG_E_HIP;
    size_t pi = 0;
    for (int l = 0; l < NL; ++l) {
        const LayerDef& d = LAYERS[l];
        const LayerOff& o = S.L[l];
        const float* W = (const float*)(host.data() + (grads ? o.gW : o.W));
        const float* b = (const float*)(host.data() + (grads ? o.gb : o.b));
        for (int co = 0; co < d.cout; ++co)
            for (int t1 = 0; t1 < 3; ++t1)
                for (int t2 = 0; t2 < 3; ++t2)
                    for (int ci = 0; ci < d.cin; ++ci)
                        out[pi++] = W[(size_t)co * o.kpad + (t1 * 3 + t2) * d.s_in + ci];
        for (int co = 0; co < d.cout; ++co) out[pi++] = b[co];
    }
    return RTG_OK;
}

int rtg_cnn_export(const void* state, float* params, void* stream) {
    if (!state || !params) return RTG_E_ARG;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return RTG_E_HIP;
    return export_arrays(state, params, false);
}

int rtg_cnn_read_gradients(const void* state, float* grads, void* stream) {
    if (!state || !grads) return RTG_E_ARG;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return RTG_E_HIP;
    return export_arrays(state, grads, true);
}

int rtg_cnn_forward(const void* state, const float* C, int N, int I1, int I2, float* X0, void* ws,
                    size_t ws_bytes, void* stream) {
    if (!state || !C || !X0 || !ws) return RTG_E_ARG;
    if (check_dims(N, I1, I2)) return RTG_E_SHAPE;
    const WsLayout W = ws_layout(N, I1, I2);
    if (ws_bytes < W.total) return RTG_E_WORKSPACE;
    const StateLayout S = state_layout();
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    char* st = (char*)state;
    const size_t px = (size_t)N * I1 * I2;
    hipLaunchKernelGGL(k_pack, dim3((px + 255) / 256), dim3(256), 0, s, C, N, I1, I2, (bf16_t*)(w + W.xin));
    // three fused pairs of layers: (0, 1), (2, 3), (4, 5)
    const int ntiles = N * ((I2 + C2_TH - 1) / C2_TH) * ((I1 + C2_TW - 1) / C2_TW);
    const int grid = std::min(ntiles, C2_MAX_WG);
    auto pair = [&](int l, const bf16_t* x, bf16_t* out) {
        Conv2Args a{};
        a.N = N; a.I1 = I1; a.I2 = I2;
        a.x = x;
        a.wA = (const bf16_t*)(st + S.L[l].Wh);
        a.bA = (const float*)(st + S.L[l].b);
        a.wB = (const bf16_t*)(st + S.L[l + 1].Wh);
        a.bB = (const float*)(st + S.L[l + 1].b);
        a.out = out;
        a.C = C;
        a.X0 = X0;
        return a;
    };
    bf16_t* h0 = (bf16_t*)(w + W.act[0]);
    bf16_t* h1 = (bf16_t*)(w + W.act[1]);
    if (conv2<8, 32, 32, false>(pair(0, (const bf16_t*)(w + W.xin), h0), grid, s) != hipSuccess ||
        conv2<32, 32, 32, false>(pair(2, h0, h1), grid, s) != hipSuccess ||
        conv2<32, 16, 8, true>(pair(4, h1, nullptr), grid, s) != hipSuccess)
        return RTG_E_HIP;
    return RTG_OK;
}

int rtg_cnn_gradients(void* state, const float* C, const float* Y, int N, int I1, int I2, void* ws,
                      size_t ws_bytes, float* loss, void* stream) {
    if (!state || !C || !Y || !ws || !loss) return RTG_E_ARG;
    if (check_dims(N, I1, I2)) return RTG_E_SHAPE;
    const WsLayout W = ws_layout(N, I1, I2);
    if (ws_bytes < W.total) return RTG_E_WORKSPACE;
    const StateLayout S = state_layout();
    hipStream_t s = (hipStream_t)stream;
    char* w = (char*)ws;
    char* st = (char*)state;
    const size_t px = (size_t)N * I1 * I2;
    const float gscale = 2.0f / (float)(px * 3);
    hipLaunchKernelGGL(k_pack, dim3((px + 255) / 256), dim3(256), 0, s, C, N, I1, I2, (bf16_t*)(w + W.xin));
    // forward, keeping every hidden activation
    const bf16_t* acts[NL];
    acts[0] = (const bf16_t*)(w + W.xin);
    for (int l = 0; l < NL; ++l) {
        bf16_t* out = l < NL - 1 ? (bf16_t*)(w + W.act[l]) : (bf16_t*)(w + W.g8);
        if (layer_forward(l, st, S, acts[l], out, C, Y, nullptr, (float*)(w + W.loss), gscale, N, I1, I2,
                          W.nconv, true, s) != hipSuccess)
            return RTG_E_HIP;
        if (l < NL - 1) acts[l + 1] = out;
    }
    // loss = mean squared error (sum of per-workgroup partials / elements)
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(64), 0, s, (const float*)(w + W.loss), W.nconv, 1, loss);
    // backward
    const bf16_t* g = (const bf16_t*)(w + W.g8);
    for (int l = NL - 1; l >= 0; --l) {
        const LayerOff& o = S.L[l];
        WgradArgs wa{N, I1, I2, WG_ROWS, g, acts[l], (float*)(w + W.part)};
        hipError_t e;
        if (l == 0) e = wgrad<8, 32, 32>(wa, W.nwg, s);
        else if (l < NL - 1) e = wgrad<32, 32, 32>(wa, W.nwg, s);
        else e = wgrad<32, 8, 16>(wa, W.nwg, s);
        if (e != hipSuccess) return RTG_E_HIP;
        const int len = o.nw + o.nb;
        hipLaunchKernelGGL(k_reduce_parts, dim3((len + 255) / 256), dim3(256), 0, s, (const float*)(w + W.part),
                           W.nwg, len, (float*)(st + o.gW));
        if (l > 0) {
            // gradient w.r.t. the layer input, masked by the ReLU of that input
            ConvArgs a{};
            a.N = N; a.I1 = I1; a.I2 = I2;
            a.x = g;
            a.w = (const bf16_t*)(st + o.Wt);
            a.mask = acts[l];
            bf16_t* gout = (bf16_t*)(w + ((l % 2) ? W.gA : W.gB));
            a.out = gout;
            if (l == NL - 1) e = conv<8, 32, 32, CV_BWD_DATA>(a, W.nconv, s);
            else e = conv<32, 32, 32, CV_BWD_DATA>(a, W.nconv, s);
            if (e != hipSuccess) return RTG_E_HIP;
            g = gout;
        }
    }
    return hipGetLastError() == hipSuccess ? RTG_OK : RTG_E_HIP;
}

int rtg_cnn_adam(void* state, float lr, int step, void* stream) {
    if (!state || step < 1) return RTG_E_ARG;
    const StateLayout S = state_layout();
    hipStream_t s = (hipStream_t)stream;
    char* st = (char*)state;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    for (int l = 0; l < NL; ++l) {
        const LayerDef& d = LAYERS[l];
        const LayerOff& o = S.L[l];
        hipLaunchKernelGGL(k_adam, dim3((o.nw + 255) / 256), dim3(256), 0, s, (float*)(st + o.W), (float*)(st + o.mW),
                           (float*)(st + o.vW), (const float*)(st + o.gW), o.nw, lr, b1, b2, eps, c1, c2);
        hipLaunchKernelGGL(k_adam, dim3(1), dim3(64), 0, s, (float*)(st + o.b), (float*)(st + o.mb),
                           (float*)(st + o.vb), (const float*)(st + o.gb), o.nb, lr, b1, b2, eps, c1, c2);
        const int n = std::max(o.nw, 32 * o.kpad_t);
        hipLaunchKernelGGL(k_make_weights, dim3((n + 255) / 256), dim3(256), 0, s, (const float*)(st + o.W),
                           d.cout_m, o.kpad, d.s_in, (bf16_t*)(st + o.Wh), l > 0 ? (bf16_t*)(st + o.Wt) : nullptr,
                           d.s_out, o.kpad_t);
    }
    return hipGetLastError() == hipSuccess ? RTG_OK : RTG_E_HIP;
}

}  // extern "C"
