#pragma once
// Banded Einstein-product operator (eq. (2); Sec. 5.1-5.2):
//
//   Y[i1,i2,j] = sum_k B[k,j] sum_{k2} A2[i2,k2] sum_{k1} A1[i1,k1] X[k1,k2,k]
//             = (X x_1 A1 x_2 A2 x_3 B^T)[i1,i2,j],
//
// with A1, A2, B banded (half-bandwidths r1, r2, rB) and zero boundary
// conditions.  Mode products on different modes commute, so each input
// channel k is blurred spatially once and scattered into the (at most
// 2 rB + 1) output channels it feeds.
//
// Tile: 64 rows (i1) x 32 columns (i2) x up to JT (4 or 8) output channels.  For every
// input channel the workgroup stages a (64 + 2R) x (32 + 2R) slab in LDS
// (zeros outside the image), runs the i1 pass with lanes across columns
// (band coefficients are wave-uniform), then the i2 pass with lanes across
// rows (again wave-uniform coefficients), and accumulates B-weighted results
// in registers.  Global loads and stores run along i1, the contiguous mode.
// R (a template tier 4/8/12) bounds r1, r2; actual widths are runtime.
//
// General PSF with float32 input of at most three channels (DMA): the slabs
// of all input channels of the tile are requested at once by asynchronous
// global-to-LDS loads of 16-byte chunks along i1, so their latencies overlap
// instead of following one another; chunks outside the image (always whole
// chunks: I1 and the tile origins are multiples of 4) are fetched from past
// the buffer range and read as zeros.  A slab column holds an odd number of
// chunks, so that 16-byte LDS reads with lanes across columns are free of
// bank conflicts.  (Measured: 58.8 -> 48.3 us per launch of the 9x9 PSF on
// 16 x 512x512x3.  The separable passes measured no faster this way, 65 us
// against 61 us at two instead of three workgroups per CU.)  Other float32
// input below 2^31 bytes is staged through registers in the same 16-byte
// chunks and layout by buffer loads that read zeros past the range (one
// load and one LDS write per four values: the single-word staging's index
// arithmetic had made the kernel VALU-bound); bfloat16 input and larger
// tensors keep single-word staging.  Coefficient rows are padded to
// multiples of 4 floats and read from LDS 16 bytes at a time; Toeplitz bands
// (TP) keep their taps in wave-uniform registers instead (counters had
// shown 22% of wave cycles waiting to issue LDS instructions, most of them
// coefficient reads: 49.1 -> 36.1 us per separable launch).
//
// General (non-separable) PSF (eqs. (56)-(57)): with ST the two passes are
// replaced by the 2-D stencil
//   U[i1,i2] = sum_{a,b} St[a,b] X_k[i1 + a, i2 + b],  |a|, |b| <= r,
// St the PSF rotated by 180 degrees (the weight of each shifted pixel), read
// from LDS as wave-uniform broadcasts; lane = row, eight columns per lane,
// one slab row (8 + 2R columns) in registers per stencil row.

#include "rtg_internal.h"

namespace rtg {

struct PhiArgs {
    int I1, I2, J, r1, r2, rB;
    const float* a1;
    const float* a2;
    const float* bb;
    const void* src;
    const float* C;   // residual mode when non-null: Y = C - Phi(X)
    float* dst;
    const float* st;  // stencil ((2 r1 + 1)^2, [a + r1][b + r1]) of a general PSF, else null
    const float* taps;  // Toeplitz bands (convolutions): A1 taps at [r1 + dd], A2 taps at
                        // [2 RMAX_SPATIAL + 1 + r2 + dd]; null for general bands
    bf16_t* dst_bf;     // non-null: the result goes there, rounded to bfloat16, instead of dst
};

__device__ __forceinline__ int xcd_remap(int b, int G) {
    // Consecutive workgroups are dispatched round-robin over the 8 XCDs;
    // remap so that each XCD receives a contiguous range of logical tiles
    // (neighbouring tiles share halos through that XCD's L2).
    const int X = 8;
    int x = b % X, slot = b / X;
    int q = G / X, rem = G % X;
    return x * q + min(x, rem) + slot;
}

// slab staging: SL_SCALAR (single-word loads through registers; bfloat16
// input, tensors of 2^31 bytes or more), SL_VEC (16-byte buffer loads through
// registers), SL_DMA (asynchronous global-to-LDS loads, general PSF)
enum { SL_SCALAR = 0, SL_VEC = 1, SL_DMA = 2 };

template <int R, int JT, int SL>
struct PhiLayout {
    static constexpr int T1 = PHI_T1, T2 = PHI_T2;
    static constexpr int SR = T1 + 2 * R;                 // slab rows
    static constexpr int SC = T2 + 2 * R;                 // slab columns (<= 64)
    static constexpr int CPC = ((SR / 4) % 2 == 0) ? SR / 4 + 1 : SR / 4;   // 16-byte chunks: odd per column
    static constexpr int SRP = SL != SL_SCALAR ? 4 * CPC : SR + 1;          // slab column stride (floats)
    static constexpr int NBUF = SL == SL_DMA ? 3 : 1;     // slabs in LDS (DMA: every input channel, J <= 3)
    static constexpr int ZRP = T1 + 1;
    static constexpr int WP = ((2 * R + 1) + 3) / 4 * 4;  // padded taps per band row
    static constexpr int NKB = JT + 2 * RMAX_B;           // input channels per tile (max)
    static constexpr int FLOATS = NBUF * SC * SRP + SC * ZRP + (T1 + T2) * WP + NKB * JT;
};

// TP: Toeplitz bands (the blurs of Sec. 5 are convolutions): the taps are
// held in wave-uniform registers for the whole tile instead of a
// coefficient row per output row and column read from LDS.
template <int R, bool BF16IN, int JT, bool ST, int SL, bool TP>
__device__ __forceinline__ void phi_tile(const PhiArgs& a, int tile, float* smem) {
    static_assert(!(TP && ST), "Toeplitz taps are for separable bands");
    constexpr bool DMA = SL == SL_DMA, VEC = SL != SL_SCALAR;
    static_assert(!(VEC && BF16IN), "16-byte slab loads take float32 input");
    static_assert(!DMA || JT == 4, "asynchronous slab loads: one tile holds every channel (J <= 3)");
    typedef float f4v __attribute__((ext_vector_type(4)));
    using LY = PhiLayout<R, JT, SL>;
    constexpr int T1 = PHI_T1, T2 = PHI_T2;
    constexpr int SR = LY::SR, SC = LY::SC, SRP = LY::SRP, NBUF = LY::NBUF, CPC = LY::CPC;
    constexpr int ZRP = LY::ZRP, WP = LY::WP, NKB = LY::NKB;
    float* Sall = smem;                  // NBUF x [SC][SRP]
    float* Z = Sall + NBUF * SC * SRP;   // [SC][ZRP]
    static_assert((NBUF * SC * SRP + SC * ZRP) % 4 == 0, "coefficient rows start 16-byte aligned");
    float* A1c = Z + SC * ZRP;           // [T1][WP]: A1[i1, i1 + d], d = t - R (0 outside the band)
    float* Stc = A1c;                    // ST: [2R + 1][WP] stencil rows (fit in T1 WP floats)
    float* A2c = A1c + T1 * WP;          // [T2][WP]
    float* Bc = A2c + T2 * WP;           // [NKB][JT]: B[k, j0 + jj]

    const int I1 = a.I1, I2 = a.I2, J = a.J;
    const int nt1 = (I1 + T1 - 1) / T1, nt2 = (I2 + T2 - 1) / T2;
    const int t1 = tile % nt1;
    const int rest = tile / nt1;
    const int t2 = rest % nt2;
    const int tj = rest / nt2;
    const int i10 = t1 * T1, i20 = t2 * T2, j0 = tj * JT;
    const int jn = min(JT, J - j0);
    const int r1 = a.r1, r2 = a.r2, rB = a.rB;
    const int w1 = 2 * r1 + 1, w2 = 2 * r2 + 1, wB = 2 * rB + 1;
    const int klo = max(0, j0 - rB), khi = min(J, j0 + jn + rB);

    const int tid = block_tid();
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const size_t plane = (size_t)I1 * I2;
    const int nk = khi - klo;

    // DMA: slab of input channel k into buffer b (chunk c: column c / CPC,
    // rows 4 (c % CPC) .. + 3; the last chunk of a column is padding)
    const auto rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.src), (short)0,
                                                        VEC ? (int)(plane * (size_t)J * 4) : 0, 0x00020000);
    auto dma_slab = [&](int k, int b) {
        float* Sd = Sall + b * SC * SRP;
        constexpr int NCH = SC * CPC;
#pragma unroll
        for (int it = 0; it < (NCH + 255) / 256; ++it) {
            const int c = it * 256 + tid;
            if (c < NCH) {
                const int col = c / CPC, rc = c % CPC;
                const int i1 = i10 - R + 4 * rc, i2 = i20 - R + col;
                const bool ok = (rc < SR / 4) & (i1 >= 0) & (i1 < I1) & (i2 >= 0) & (i2 < I2);
                const unsigned off = ok ? (unsigned)(((size_t)k * plane + (size_t)i2 * I1 + i1) * 4) : 0x80000000u;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rsrc, (__attribute__((address_space(3))) void*)(Sd + (size_t)(it * 256 + wave * 64) * 4), 16, off, 0,
                    0, 0);
            }
        }
    };
    if constexpr (DMA) {
        for (int kk = 0; kk < nk; ++kk) dma_slab(klo + kk, kk);     // nk <= J <= 3 = NBUF
    }

    // band coefficients of this tile, zero-padded to R taps and to rows of
    // WP (a multiple of 4) floats: the passes read them as 16-byte LDS
    // broadcasts, four taps a read, with no branches
    if constexpr (ST) {
        static_assert((2 * R + 1) * WP <= T1 * WP, "stencil fits the band-coefficient area");
        for (int e = tid; e < (2 * R + 1) * WP; e += 256) {
            const int da = e / WP - R, db = e % WP - R;
            Stc[e] = (db <= R && da >= -r1 && da <= r1 && db >= -r1 && db <= r1)
                         ? a.st[(size_t)(da + r1) * w1 + db + r1]
                         : 0.f;
        }
    } else if constexpr (!TP) {
        for (int e = tid; e < T1 * WP; e += 256) {
            const int row = e / WP, t = e % WP, dd = t - R;
            const int i1 = i10 + row;
            A1c[e] = (t <= 2 * R && dd >= -r1 && dd <= r1 && i1 < I1) ? a.a1[(size_t)i1 * w1 + r1 + dd] : 0.f;
        }
        for (int e = tid; e < T2 * WP; e += 256) {
            const int col = e / WP, t = e % WP, dd = t - R;
            const int i2 = i20 + col;
            A2c[e] = (t <= 2 * R && dd >= -r2 && dd <= r2 && i2 < I2) ? a.a2[(size_t)i2 * w2 + r2 + dd] : 0.f;
        }
    }
    for (int e = tid; e < NKB * JT; e += 256) {
        const int kk = e / JT, jj = e % JT;
        const int k = klo + kk, j = j0 + jj, dd = j - k;
        Bc[e] = (k < khi && jj < jn && dd >= -rB && dd <= rB) ? a.bb[(size_t)k * wB + dd + rB] : 0.f;
    }

    float acc[JT][8];
#pragma unroll
    for (int jj = 0; jj < JT; ++jj)
#pragma unroll
        for (int o = 0; o < 8; ++o) acc[jj][o] = 0.f;
    float tA1[WP], tA2[WP];                 // TP: the taps, zero past the band
    if constexpr (TP) {
#pragma unroll
        for (int t = 0; t < WP; ++t) {
            const int dd = t - R;
            const float v1 = (t <= 2 * R && dd >= -r1 && dd <= r1) ? *gptr(a.taps + r1 + dd) : 0.f;
            const float v2 = (t <= 2 * R && dd >= -r2 && dd <= r2) ? *gptr(a.taps + 2 * RMAX_SPATIAL + 1 + r2 + dd) : 0.f;
            tA1[t] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v1)));
            tA2[t] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v2)));
        }
    }
    // one padded coefficient row from LDS, 16 bytes a read (rows start at
    // multiples of 4 floats of a 16-byte aligned area)
    auto load_row = [](const float* row, float (&cf)[WP]) {
#pragma unroll
        for (int q = 0; q < WP / 4; ++q) {
            const f4v v = *(const f4v*)(row + 4 * q);
#pragma unroll
            for (int i = 0; i < 4; ++i) cf[4 * q + i] = v[i];
        }
    };

    // Register staging: the slab of the next input channel is loaded into
    // registers while the current one is processed (all loads of a slab are
    // issued together).
    constexpr int NLD = VEC ? 1 : (SR * SC + 255) / 256;
    // SL_VEC: the slab in 16-byte chunks (the layout of the asynchronous
    // loads), zeros past the buffer range
    constexpr int NCHV = SC * CPC;
    constexpr int NLD4 = (SL == SL_VEC) ? (NCHV + 255) / 256 : 1;
    f4v pre4[NLD4];
    auto load_slab4 = [&](int k) {
#pragma unroll
        for (int it = 0; it < NLD4; ++it) {
            const int c = it * 256 + tid;
            const int col = c / CPC, rc = c % CPC;
            const int i1 = i10 - R + 4 * rc, i2 = i20 - R + col;
            const bool ok = (c < NCHV) & (rc < SR / 4) & (i1 >= 0) & (i1 < I1) & (i2 >= 0) & (i2 < I2);
            const unsigned off = ok ? (unsigned)(((size_t)k * plane + (size_t)i2 * I1 + i1) * 4) : 0x80000000u;
            pre4[it] = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0));
        }
    };
    const float* srcf = (const float*)a.src;
    const bf16_t* srch = (const bf16_t*)a.src;
    float pre[NLD];
    auto load_slab = [&](int k) {
#pragma unroll
        for (int it = 0; it < NLD; ++it) {
            // unconditional load from a clamped address, masked afterwards
            const int e = tid + 256 * it;
            const int row = e % SR, c = e / SR;
            const int i1 = i10 - R + row, i2 = i20 - R + c;
            const bool inb = e < SR * SC && i1 >= 0 && i1 < I1 && i2 >= 0 && i2 < I2;
            const size_t off = (size_t)k * plane + (size_t)min(max(i2, 0), I2 - 1) * I1 + min(max(i1, 0), I1 - 1);
            const float v = BF16IN ? bf2f(*gptr(srch + off)) : *gptr(srcf + off);
            pre[it] = inb ? v : 0.f;
        }
    };
    if constexpr (SL == SL_VEC) load_slab4(klo);
    else if constexpr (SL == SL_SCALAR) load_slab(klo);
    for (int kk = 0; kk < nk; ++kk) {
        const int k = klo + kk;
        float* S = Sall + (kk % NBUF) * SC * SRP;
        if constexpr (DMA) {
            // every slab was requested before the coefficients were staged
            if (kk == 0) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's loads landed
            __syncthreads();                                    // everyone's; Z free
        } else if constexpr (SL == SL_VEC) {
            __syncthreads();
#pragma unroll
            for (int it = 0; it < NLD4; ++it) {
                const int c = it * 256 + tid;
                if (c < NCHV) *(f4v*)(S + 4 * c) = pre4[it];   // column c / CPC, rows 4 (c % CPC) ..
            }
            if (k + 1 < khi) load_slab4(k + 1);
            __syncthreads();
        } else {
            __syncthreads();
            // ---- stage the slab of channel k (zero boundary conditions)
#pragma unroll
            for (int it = 0; it < NLD; ++it) {
                const int e = tid + 256 * it;
                if (e < SR * SC) S[(e / SR) * SRP + e % SR] = pre[it];
            }
            if (k + 1 < khi) load_slab(k + 1);
            __syncthreads();
        }
        float u[8];
        if constexpr (ST) {
            // ---- 2-D stencil: lane = row, columns 8 wave + o
#pragma unroll
            for (int o = 0; o < 8; ++o) u[o] = 0.f;
#pragma unroll
            for (int ta = 0; ta <= 2 * R; ++ta) {
                float in[8 + 2 * R];
#pragma unroll
                for (int e = 0; e < 8 + 2 * R; ++e) in[e] = S[(wave * 8 + e) * SRP + lane + ta];
                float cf[WP];
                load_row(Stc + ta * WP, cf);
#pragma unroll
                for (int o = 0; o < 8; ++o)
#pragma unroll
                    for (int tb = 0; tb <= 2 * R; ++tb) u[o] = fmaf(cf[tb], in[o + tb], u[o]);
            }
        } else {
        // ---- i1 pass: Z[c][row] = sum_d A1[i1, i1+d] S[c][row + R + d]
        // lanes across slab columns, wave handles rows [16 wave, 16 wave + 16)
        if (lane < SC) {
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                const int rbase = wave * 16 + blk * 8;
                float in[8 + 2 * R];
                if constexpr (VEC) {
#pragma unroll
                    for (int q = 0; q < (8 + 2 * R) / 4; ++q) {
                        const f4v v = *(const f4v*)(S + lane * SRP + rbase + 4 * q);
#pragma unroll
                        for (int i = 0; i < 4; ++i) in[4 * q + i] = v[i];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8 + 2 * R; ++e) in[e] = S[lane * SRP + rbase + e];
                }
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    float cf[WP];
                    if constexpr (TP) {
#pragma unroll
                        for (int t = 0; t < WP; ++t) cf[t] = tA1[t];
                    } else {
                        load_row(A1c + (rbase + o) * WP, cf);
                    }
                    float s = 0.f;
#pragma unroll
                    for (int t = 0; t <= 2 * R; ++t) s = fmaf(cf[t], in[o + t], s);
                    Z[lane * ZRP + rbase + o] = s;
                }
            }
        }
        __syncthreads();
        // ---- i2 pass: U[row][o] = sum_d A2[i2, i2+d] Z[8 wave + o + R + d][row]
        float in2[8 + 2 * R];
#pragma unroll
        for (int e = 0; e < 8 + 2 * R; ++e) in2[e] = Z[(wave * 8 + e) * ZRP + lane];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            float cf[WP];
            if constexpr (TP) {
#pragma unroll
                for (int t = 0; t < WP; ++t) cf[t] = tA2[t];
            } else {
                load_row(A2c + (wave * 8 + o) * WP, cf);
            }
            float s = 0.f;
#pragma unroll
            for (int t = 0; t <= 2 * R; ++t) s = fmaf(cf[t], in2[o + t], s);
            u[o] = s;
        }
        }   // separable passes
        // ---- mode 3: output channel j receives B[k, j] * U (|j - k| <= rB)
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
            const float bkj = Bc[(k - klo) * JT + jj];
#pragma unroll
            for (int o = 0; o < 8; ++o) acc[jj][o] = fmaf(bkj, u[o], acc[jj][o]);
        }
    }
    // ---- store (lanes along i1: coalesced).  In residual mode the values
    // of C are loaded first, all together, from clamped addresses.
    const int i1 = i10 + lane;
    const int i1c = min(i1, I1 - 1);
    float cv[JT][8];
    if (a.C) {
#pragma unroll
        for (int jj = 0; jj < JT; ++jj)
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int jc = min(j0 + jj, J - 1), i2c = min(i20 + wave * 8 + o, I2 - 1);
                cv[jj][o] = *gptr(a.C + (size_t)jc * plane + (size_t)i2c * I1 + i1c);
            }
#pragma unroll
        for (int jj = 0; jj < JT; ++jj)
#pragma unroll
            for (int o = 0; o < 8; ++o) acc[jj][o] = cv[jj][o] - acc[jj][o];
    }
    if (i1 < I1) {
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
            if (jj >= jn) break;
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int i2 = i20 + wave * 8 + o;
                if (i2 < I2) {
                    const size_t e = (size_t)(j0 + jj) * plane + (size_t)i2 * I1 + i1;
                    if (a.dst_bf) *gptr_w(a.dst_bf + e) = f2bf(acc[jj][o]);
                    else *gptr_w(a.dst + e) = acc[jj][o];
                }
            }
        }
    }
}

// One operator tile of a batch: tile b of the batch's tile index space
// (problem p holds tiles [starts[p], starts[p + 1])).
template <int R, bool BF16IN, int JT, bool ST, int SL, bool TP>
__device__ __forceinline__ void phi_batched_task(const Desc* __restrict__ descs, const int* __restrict__ starts,
                                                 int count, int src_sel, int src_index, int b, float* smem) {
    const int p = find_problem(starts, count, b);
    const Desc& d = descs[p];
    if (src_sel == PS_BASIS && d.state[ST_ACTIVE] == 0) return;
    PhiArgs a;
    a.I1 = d.I1; a.I2 = d.I2; a.J = d.J; a.r1 = d.r1; a.r2 = d.r2; a.rB = d.rB;
    a.a1 = d.a1; a.a2 = d.a2; a.bb = d.bb;
    a.st = d.st;
    a.taps = TP ? d.taps : nullptr;
    if (src_sel == PS_BASIS) {
        const size_t es = d.bf16 ? 2 : 4;
        a.src = (const char*)d.V + (size_t)src_index * d.n * es;
        a.C = nullptr;
    } else {
        if (d.X0 == nullptr) return;      // R0 = C needs no operator application
        a.src = d.X0;
        a.C = d.C;
    }
    a.dst = d.W;
    a.dst_bf = (src_sel == PS_X0_V1) ? (bf16_t*)d.V : nullptr;
    phi_tile<R, BF16IN, JT, ST, SL, TP>(a, uniform_int(b - starts[p]), smem);
}

}  // namespace rtg
