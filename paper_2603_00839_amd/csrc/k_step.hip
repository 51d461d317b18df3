// One Arnoldi step over a column tile with the operator applied on the fly,
// for a bfloat16 basis (Sec. 4.3; Phi of eq. (2)):
//
//   V_{j+1} = scale * (Phi(V_j) - sum_{i<=j} h_ij V_i),   scale = 1 / h_{j+1,j}
//
// plus the partial sketches of the stored V_{j+1} with (Om1, Om2) and with
// the composed (Om1 A1, Om2 A2), from which the next step's sketched inner
// products need S(V_{j+1}) and S(Phi(V_{j+1})).  W = Phi(V_j) is never
// stored: each workgroup recomputes it for its own tile from V_j.
//
// A workgroup owns output channel c and a strip of 32 columns (i2) over all
// I1 rows, walked in blocks of 64 rows.  Per block:
//  * the raw bfloat16 slab of V_j (the input channels of c's band; the
//    block's rows with a halo of whole 8-row chunks; the strip's columns
//    with an R-wide halo) and the block's rows of A1 reach LDS through
//    asynchronous global-to-LDS loads issued while the previous block is
//    processed.  Chunks outside the tensor are fetched from past the end of
//    the buffer range, which reads zeros (the zero boundary condition);
//  * i1 pass on MFMA: each input channel's slab is blurred along i1 (band
//    coefficients as a bfloat16 high + middle pair, float32 accumulation)
//    and mixed in with its weight, Z = sum_k B[k, c] A1 V_j[k] (mode products
//    commute), into LDS as float;
//  * i2 pass: a lane per row blurs eight columns of Z, which leaves the W
//    tile in registers in the basis' own layout (lane = row);
//  * multi-AXPY with V_1..V_j (two terms in flight), scale, round to
//    bfloat16, store V_{j+1}; the tile also goes to LDS column-major;
//  * mode-1 contraction of the block on MFMA (16x16x32 bf16) against the
//    stacked rows [Om1 ; Om1 A1] (the composed matrix split into high and
//    low bfloat16 parts).
// After the last block the mode-2 contraction with Om2 / Om2 A2 writes two
// l1 x l2 partials per tile, which the sketched-Gram kernel reduces; for
// l2 <= 64 the wave's Om2 columns are requested before the mode-1 results
// go to LDS.
#include "rtg_internal.h"

namespace rtg {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int STEP_T1 = 64;                 // rows per block
constexpr int STEP_NKR = 3;                 // input channels per raw slab
constexpr int STEP_PF = 4;                  // basis terms of a block requested before the operator is applied
// Byte offset that lies past every buffer range used here: the host only
// launches this kernel when a basis vector is under 2^31 bytes.
constexpr unsigned STEP_OOB = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t step_rsrc(const void* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

#define RTG_LDS __attribute__((address_space(3)))

template <int R, int RPW>
struct StepSmem {
    static constexpr int T1 = STEP_T1, TC = TILE_TC;
    static constexpr int R8 = (R + 7) / 8 * 8;          // row halo in whole 16-byte chunks
    static constexpr int SR = T1 + 2 * R8;              // slab rows
    static constexpr int CHR = SR / 8;                  // chunks per raw column
    static constexpr int CHP = CHR | 1;                 // column stride in chunks (odd: no bank conflicts)
    static constexpr int SC = TC + 2 * R;               // slab columns
    static constexpr int NT = (SC + 15) / 16;           // column tiles of the i1 product
    static constexpr int NKB = (15 + R8 + R) / 32 + 1;  // 32-row K-blocks per 16-row tile of the i1 product
    static constexpr int NSLOT = STEP_NKR * SC * CHP;   // 16-byte slots of the raw slab
    static constexpr int RAWB = NSLOT * 16;
    static constexpr int ZRP = T1 + 4;                  // Z column stride (16-byte aligned)
    static constexpr int WP = ((2 * R + 1) + 3) / 4 * 4;
    static constexpr int XP = T1 + 8;
    static constexpr int WTP = T1 + 4;                  // stride of the transposed W tile
    static constexpr int YP = TC + 1;
    static constexpr int YB = 64 * RPW * YP * 4;
    static constexpr int UB = RAWB > YB ? RAWB : YB;
};

// TOEP: both spatial bands are Toeplitz on their in-range entries (a
// convolution with zero boundary conditions, as for the blurs of Sec. 5).
// The i1 product's coefficient fragments are then the same for every block
// (computed once per workgroup) and the i2 pass reads each group of four
// taps once for all eight outputs of a lane; otherwise the block's band rows
// are streamed into LDS and the fragments are formed per block.  Outputs of
// rows past I1 come out nonzero in either form; they are never stored.
template <int R, int RPW, bool TOEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_step(const Desc* __restrict__ descs, const int* __restrict__ starts,
                                              int count, int j) {
    using SM = StepSmem<R, RPW>;
    constexpr int T1 = SM::T1, TC = SM::TC, R8 = SM::R8, SR = SM::SR, CHR = SM::CHR, CHP = SM::CHP, SC = SM::SC;
    constexpr int NT = SM::NT, NKB = SM::NKB;
    constexpr int NSLOT = SM::NSLOT, ZRP = SM::ZRP, WP = SM::WP, XP = SM::XP, WTP = SM::WTP, YP = SM::YP;
    constexpr int NKR = STEP_NKR;
    constexpr int NIN = 8 + 2 * R;                      // i2-pass window (columns) per eight outputs

    // Separate LDS arrays: reads of one are not held back by the compiler
    // for asynchronous loads still in flight into another.
    __shared__ float coef_s[MMAX + 2];
    __shared__ float bw_s[2 * RMAX_B + 1];              // B[k, c] for the input channels klo .. khi - 1
    __shared__ __attribute__((aligned(16))) unsigned char su[SM::UB];
    __shared__ __attribute__((aligned(16))) float Z[SC * ZRP];    // [col][row] after the i1 product
    __shared__ __attribute__((aligned(16))) float Wt[TC * WTP];   // [col][row]: the W tile, for the multi-AXPY
    __shared__ __attribute__((aligned(16))) float A1c[TOEP ? WP : T1 * WP];   // TOEP: the taps of A1
    __shared__ __attribute__((aligned(16))) float A2c[TOEP ? WP : TC * WP];   // TOEP: the taps of A2
    __shared__ __attribute__((aligned(16))) bf16_t Xh[TC * XP];
    bf16_t* raw = (bf16_t*)su;                          // slot s = (kk SC + col) CHP + rc: rows 8 rc .. 8 rc + 7
    float* Ys = (float*)su;                             // mode-1 results (after the last block)

    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int p = find_problem(starts, count, b);
    const Desc& d = descs[p];
    const int tile = uniform_int(b - starts[p]);
    if (d.state[ST_ACTIVE] == 0) return;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m16 = lane & 15, kq = lane >> 4;
    const int I1 = d.I1, I2 = d.I2, J = d.J;
    const int l1 = d.l1, l2 = d.l2;
    const int t2 = tile % d.n_i2t, c = tile / d.n_i2t;
    const int i20 = t2 * TC;
    const int ncol = min(TC, I2 - i20);
    const int r2 = d.r2, rB = d.rB;
    const int w2 = 2 * r2 + 1, wB = 2 * rB + 1;
    const int klo = max(0, c - rB), khi = min(J, c + rB + 1);
    const unsigned plane = (unsigned)I1 * (unsigned)I2;
    const size_t tile_off = (size_t)c * plane + (size_t)i20 * I1;
    const int tile_elems = ncol * I1;
    const auto rvj = step_rsrc((const bf16_t*)d.V + (size_t)(j - 1) * d.n, (int)(d.n * 2));   // V_j
    const float* a1p = d.a1p[R == 4 ? 0 : (R == 8 ? 1 : 2)];
    // Om1 and the composed Om1 A1 (high plane, then low plane) in operand order
    const int nkbf = frag_nkb(I1, FRAG_K_BF16);
    const unsigned om1_lo = (unsigned)frag_elems(l1, I1, FRAG_K_BF16) * 2u;
    const auto rom1 = step_rsrc(d.om1hf, (int)om1_lo);
    const auto rom1c = step_rsrc(d.om1th, 2 * (int)om1_lo);

    const int nterms = j;
    for (int i = tid; i < nterms; i += 256) coef_s[i] = d.coef[i];
    if (tid < khi - klo) bw_s[tid] = *gptr(d.bb + (size_t)(klo + tid) * wB + rB + (c - klo - tid));
    const float scale = d.coef[MMAX + 1];
    if constexpr (TOEP) {
        if (tid < WP) {
            const int dd = tid - R, r1 = d.r1;
            A1c[tid] = (tid <= 2 * R && dd >= -r1 && dd <= r1) ? *gptr(d.taps + r1 + dd) : 0.f;
            A2c[tid] = (tid <= 2 * R && dd >= -r2 && dd <= r2) ? *gptr(d.taps + 2 * RMAX_SPATIAL + 1 + r2 + dd) : 0.f;
        }
    } else {
        for (int e = tid; e < TC * WP; e += 256) {
            const int col = e / WP, t = e % WP, dd = t - R;
            const int i2 = i20 + col;
            A2c[e] = (t <= 2 * R && dd >= -r2 && dd <= r2 && i2 < I2) ? *gptr(d.a2 + (size_t)i2 * w2 + r2 + dd)
                                                                        : 0.f;
        }
    }

    const int RT = (l1 + 15) >> 4;
    const int NRT = 2 * RT;
    f4 acc[RPW][2];
#pragma unroll
    for (int u = 0; u < RPW; ++u)
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[u][g] = f4{0.f, 0.f, 0.f, 0.f};

    // Asynchronous loads into LDS: a wave's instruction fills a 1 KB window,
    // lane i writing bytes 16 i .. 16 i + 15 of it, so slot s is fetched by
    // thread s % 256 of pass s / 256.
    auto dma_slab = [&](int rb, int k0) {
        const int i10 = rb * T1;
        auto one = [&](int it) {
            const int s = it * 256 + tid;
            const int kk = s / (SC * CHP), rem = s % (SC * CHP);
            const int col = rem / CHP, rc = rem % CHP;
            const int k = k0 + kk, i1 = i10 - R8 + 8 * rc, i2 = i20 - R + col;
            // I1 is a multiple of 8: a chunk is wholly inside the tensor or wholly outside
            const bool ok = (rc < CHR) & (k < khi) & (i1 >= 0) & (i1 < I1) & (i2 >= 0) & (i2 < I2);
            const unsigned off = ok ? ((unsigned)k * plane + (unsigned)i2 * (unsigned)I1 + (unsigned)i1) * 2u
                                    : STEP_OOB;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rvj, (RTG_LDS void*)(raw + (it * 256 + wave * 64) * 8), 16, off,
                                                     0, 0, 0);
        };
#pragma unroll
        for (int it = 0; it < NSLOT / 256; ++it) one(it);
        if constexpr (NSLOT % 256 != 0)
            if (tid < NSLOT % 256) one(NSLOT / 256);
    };
    auto dma_bands = [&](int rb) {
        const int i10 = rb * T1;
        // rows i10 .. i10 + 63 of the padded band copy; rows past I1 read zeros
        const auto ra = step_rsrc(a1p + (size_t)i10 * WP, (I1 - i10) * WP * 4);
        constexpr int NA = T1 * WP / 4;
        auto one = [&](int it) {
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (RTG_LDS void*)(A1c + (it * 256 + wave * 64) * 4), 16,
                                                     (unsigned)(it * 256 + tid) * 16u, 0, 0, 0);
        };
#pragma unroll
        for (int it = 0; it < NA / 256; ++it) one(it);
        if constexpr (NA % 256 != 0)
            if (tid < NA % 256) one(NA / 256);
    };
    // the channel weights come from LDS: a vector-memory load here would make
    // the i1 pass wait for every load issued before it (the counter runs in
    // issue order), the block's basis terms included
    auto bweight = [&](int k) { return k < khi ? bw_s[k - klo] : 0.f; };

    // ---- the i1 product on MFMA.  Wave w owns output rows 16 w .. 16 w + 15
    // of every block; their inputs are slab rows [16 w + R8 - R, 16 w + 15 +
    // R8 + R], covered by NKB K-blocks of 32 rows starting at kstart(q)
    // (clamped to the slab; rows an earlier K-block covers get coefficient
    // zero).  A operand: the A1 coefficient of output row 16 w + m16 and slab
    // row kstart(q) + 8 kq + e, split into two bfloat16 terms (high and
    // middle: their sum is the float32 coefficient to about 2^-17 of its
    // size, far below the bfloat16 rounding of the stored basis); B operand:
    // 8 consecutive slab rows of one column, one 16-byte LDS chunk of the raw
    // bfloat16 slab.  The products are exact and accumulate in float32.
    auto kstart = [&](int q) { return min(16 * wave + 32 * q, SR - 32); };
    u4 afr[NKB][2];
    auto make_frags = [&]() {
#pragma unroll
        for (int q = 0; q < NKB; ++q) {
            const int s0 = kstart(q);
            const int covered = q > 0 ? kstart(q - 1) + 32 : 0;   // rows below this are an earlier K-block's
            unsigned hw[4] = {0u, 0u, 0u, 0u}, mw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int sr = s0 + 8 * kq + e;
                const int orow = 16 * wave + m16;
                const int dd = sr - R8 - orow;
                const bool ok = (dd >= -R) & (dd <= R) & (sr >= covered);
                const int tix = min(max(dd + R, 0), 2 * R);
                float cf;
                if constexpr (TOEP) cf = A1c[tix];
                else cf = A1c[orow * WP + tix];
                cf = ok ? cf : 0.f;
                const bf16_t h = f2bf(cf);
                const float r1v = cf - bf2f(h);
                const bf16_t mm = f2bf(r1v);
                const int sh = (e & 1) * 16;
                hw[e >> 1] |= (unsigned)h << sh;
                mw[e >> 1] |= (unsigned)mm << sh;
            }
            afr[q][0] = u4{hw[0], hw[1], hw[2], hw[3]};
            afr[q][1] = u4{mw[0], mw[1], mw[2], mw[3]};
        }
    };
    if constexpr (TOEP) {
        __syncthreads();                                   // taps in LDS
        make_frags();
    }

    const int nrb = (I1 + T1 - 1) / T1;
    dma_slab(0, klo);
    if constexpr (!TOEP) dma_bands(0);
    // the multi-AXPY's share of a thread: eight consecutive rows of one
    // column of the block (16-byte accesses)
    const int acol = tid >> 3, arow = 8 * (tid & 7);
    auto load_term = [&](int i, unsigned aoff) {
        const auto rv = step_rsrc((const bf16_t*)d.V + (size_t)i * d.n + tile_off, tile_elems * 2);
        return __builtin_amdgcn_raw_buffer_load_b128(rv, aoff, 0, 0);
    };
    for (int rb = 0; rb < nrb; ++rb) {
        const int i10 = rb * T1;
        const bool aok = (i10 + arow < I1) & (acol < ncol);
        const unsigned aoff = aok ? (unsigned)(acol * I1 + i10 + arow) * 2u : STEP_OOB;
        // the block's first STEP_PF basis terms are requested now, so that they
        // arrive while the operator is applied
        // Wave priorities (s_setprio) among the three workgroups of a CU: a
        // wave issuing its memory requests goes first (2), so that their
        // latency starts early; a wave in a run of matrix products next (1);
        // the rest at 0.
        u4 pre[STEP_PF];
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int i = 0; i < STEP_PF; ++i) pre[i] = i < nterms ? load_term(i, aoff) : u4{0u, 0u, 0u, 0u};
        __builtin_amdgcn_s_setprio(0);
        // ---- i1 product over groups of NKR input channels, each channel's
        // product mixed in with its weight B[k, c] (mode products commute):
        //      Z[col][row] = sum_k B[k, c] sum_i' A1[i1, i'] V_j[k][i'][col]
        f4 zacc[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) zacc[n] = f4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = klo; k0 < khi; k0 += NKR) {
            if (k0 > klo) {
                __syncthreads();                           // previous group's slab reads done
                dma_slab(rb, k0);
            }
            // this wave's loads into LDS have landed once at most nv younger
            // vector-memory instructions are outstanding (the counter runs in
            // issue order): the basis terms requested above and, after the
            // first block, the previous block's store stay in flight
            const int nv = (k0 > klo) ? 0 : (rb > 0 ? 1 : 0) + min(nterms, STEP_PF);
            switch (nv) {
                case 0: __builtin_amdgcn_s_waitcnt(0x0F70); break;
                case 1: __builtin_amdgcn_s_waitcnt(0x0F71); break;
                case 2: __builtin_amdgcn_s_waitcnt(0x0F72); break;
                case 3: __builtin_amdgcn_s_waitcnt(0x0F73); break;
                case 4: __builtin_amdgcn_s_waitcnt(0x0F74); break;
                default: __builtin_amdgcn_s_waitcnt(0x0F75); break;
            }
            __syncthreads();
            if constexpr (!TOEP)
                if (k0 == klo) make_frags();               // this block's band rows
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int kk = 0; kk < NKR; ++kk) {
                if (k0 + kk >= khi) break;
                const float wk = bweight(k0 + kk);
                u4 bv[NKB][NT];
#pragma unroll
                for (int q = 0; q < NKB; ++q)
#pragma unroll
                    for (int n = 0; n < NT; ++n) {
                        const int colc = min(16 * n + m16, SC - 1);
                        bv[q][n] = *(const u4*)(raw + ((kk * SC + colc) * CHP + kstart(q) / 8 + kq) * 8);
                    }
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    f4 a = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int q = 0; q < NKB; ++q)
#pragma unroll
                        for (int t = 0; t < 2; ++t)
                            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, afr[q][t]),
                                                                         __builtin_bit_cast(bf8, bv[q][n]), a, 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) zacc[n][i] = fmaf(wk, a[i], zacc[n][i]);
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
        // lane: rows 16 w + 4 kq .. + 3 of slab column 16 n + m16
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int col = 16 * n + m16;
            if (col < SC) *(f4*)(Z + col * ZRP + 16 * wave + 4 * kq) = zacc[n];
        }
        __syncthreads();                                   // Z complete; slab and band rows free
        // ---- i2 pass (lane = row, eight columns per wave): the W tile
        float x[8];
        {
            float in2[NIN];
#pragma unroll
            for (int e = 0; e < NIN; ++e) in2[e] = Z[(wave * 8 + e) * ZRP + lane];
            if constexpr (TOEP) {
#pragma unroll
                for (int o = 0; o < 8; ++o) x[o] = 0.f;
#pragma unroll
                for (int t4 = 0; t4 < WP; t4 += 4) {
                    const f4 cv = *(const f4*)(A2c + t4);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (t4 + q > 2 * R) break;
#pragma unroll
                        for (int o = 0; o < 8; ++o) x[o] = fmaf(cv[q], in2[o + t4 + q], x[o]);
                    }
                }
            } else {
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const float* cr = A2c + (wave * 8 + o) * WP;
                    float s2 = 0.f;
#pragma unroll
                    for (int t = 0; t <= 2 * R; ++t) s2 = fmaf(cr[t], in2[o + t], s2);
                    x[o] = s2;
                }
            }
        }
        // ---- the W tile to LDS, read back as eight consecutive rows of one
        // column per thread: the multi-AXPY, the store and the sketch operand
        // are then 16-byte accesses
#pragma unroll
        for (int o = 0; o < 8; ++o) Wt[(wave * 8 + o) * WTP + lane] = x[o];
        u4 va = u4{0u, 0u, 0u, 0u}, vb = u4{0u, 0u, 0u, 0u};
        if (nterms > STEP_PF) va = load_term(STEP_PF, aoff);
        if (nterms > STEP_PF + 1) vb = load_term(STEP_PF + 1, aoff);
        // ---- operands of this block's mode-1 contraction (stacked rows
        // [Om1 ; Om1 A1]), requested before the stores so that they arrive
        // while the tile is stored
        const int nkb = (min(T1, I1 - i10) + 31) / 32;
        struct AF {
            u4 h, l;
        };
        // A fragments in operand order: one contiguous 1 KB read per wave and
        // tile (padding is stored zeros); the low part is fetched for the
        // composed rows only
        auto load_a = [&](int kb, AF* A) {
            const int kbg = rb * (T1 / FRAG_K_BF16) + kb;
#pragma unroll
            for (int u2 = 0; u2 < RPW; ++u2) {
                const int t = wave + 4 * u2;
                const bool half = t >= RT;
                const int tl = t - (half ? RT : 0);
                const unsigned off = (t < NRT) ? (unsigned)((tl * nkbf + kbg) * 64 + lane) * 16u : STEP_OOB;
                const auto& rs = half ? rom1c : rom1;
                A[u2].h = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
                A[u2].l = half ? __builtin_amdgcn_raw_buffer_load_b128(rs, off + om1_lo, 0, 0) : u4{0u, 0u, 0u, 0u};
            }
        };
        AF A0[RPW], A1[RPW];
        load_a(0, A0);
        if (nkb > 1) load_a(1, A1);
        __syncthreads();                                   // the W tile is in LDS
        // the next block's slab and band rows: requested here rather than
        // after the previous barrier, since a barrier's release fence makes
        // every asynchronous load to LDS still in flight land first
        __builtin_amdgcn_s_setprio(2);
        if (rb + 1 < nrb) {
            dma_slab(rb + 1, klo);
            if constexpr (!TOEP) dma_bands(rb + 1);
        }
        __builtin_amdgcn_s_setprio(0);
        float w8[8];
        {
            const f4 lo4 = *(const f4*)(Wt + acol * WTP + arow);
            const f4 hi4 = *(const f4*)(Wt + acol * WTP + arow + 4);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                w8[r] = lo4[r];
                w8[4 + r] = hi4[r];
            }
        }
        // ---- multi-AXPY, two terms in flight
        auto apply_term = [&](float ci, u4 v) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w8[2 * q] = fmaf(-ci, __uint_as_float(v[q] << 16), w8[2 * q]);
                w8[2 * q + 1] = fmaf(-ci, __uint_as_float(v[q] & 0xffff0000u), w8[2 * q + 1]);
            }
        };
#pragma unroll
        for (int i = 0; i < STEP_PF; ++i)
            if (i < nterms) apply_term(coef_s[i], pre[i]);
        for (int i = STEP_PF; i < nterms; i += 2) {
            apply_term(coef_s[i], va);
            if (i + 2 < nterms) va = load_term(i + 2, aoff);
            if (i + 1 < nterms) {
                apply_term(coef_s[i + 1], vb);
                if (i + 3 < nterms) vb = load_term(i + 3, aoff);
            }
        }
        // ---- scale, round, store V_{j+1}; the tile to LDS for the sketch
        // (zeros outside the tensor: the sketch operands' padding is zero too)
        u4 pk;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            pk[q] = (unsigned)f2bf(w8[2 * q] * scale) | ((unsigned)f2bf(w8[2 * q + 1] * scale) << 16);
        if (!aok) pk = u4{0u, 0u, 0u, 0u};
        const auto rd = step_rsrc((const bf16_t*)d.V + (size_t)j * d.n + tile_off, tile_elems * 2);
        __builtin_amdgcn_raw_buffer_store_b128(pk, rd, aoff, 0, 0);
        *(u4*)(Xh + acol * XP + arow) = pk;
        __syncthreads();
        // ---- mode-1 contraction of this block on MFMA (a block is at most two K-blocks)
        auto mfma_block = [&](int kb, const AF* A) {
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const int col = 16 * g + m16;
                const u4 bh = *(const u4*)(Xh + col * XP + kb * 32 + 8 * kq);
#pragma unroll
                for (int u2 = 0; u2 < RPW; ++u2) {
                    const int t = wave + 4 * u2;
                    if (t >= NRT) break;
                    acc[u2][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf8, A[u2].h), __builtin_bit_cast(bf8, bh), acc[u2][g], 0, 0, 0);
                    if (t >= RT)
                        acc[u2][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf8, A[u2].l), __builtin_bit_cast(bf8, bh), acc[u2][g], 0, 0, 0);
                }
            }
        };
        __builtin_amdgcn_s_setprio(1);
        mfma_block(0, A0);
        if (nkb > 1) mfma_block(1, A1);
        __builtin_amdgcn_s_setprio(0);
    }

    // ---- mode-1 results to LDS, then the mode-2 contraction
    const bool m2fast = ((l2 + 15) >> 4) == 4;
    float B0[TC / 4], B1[TC / 4];
    if (m2fast) mode2_load4<TC>(wave, lane, l2, I2, i20, ncol, NRT, RT, d.om2, d.om2t, B0, B1);
    __syncthreads();
#pragma unroll
    for (int u2 = 0; u2 < RPW; ++u2) {
        const int t = wave + 4 * u2;
        if (t >= NRT) break;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) Ys[(16 * t + 4 * kq + i) * YP + 16 * g + m16] = acc[u2][g][i];
    }
    __syncthreads();
    if (m2fast)
        mode2_partials4<TC, YP>(Ys, wave, lane, NRT, RT, l1, l2, B0, B1, d.PV + (size_t)tile * l1 * l2,
                                d.PW + (size_t)tile * l1 * l2);
    else
        mode2_partials<TC, YP>(Ys, wave, lane, NRT, RT, l1, l2, I2, i20, ncol, d.om2, d.om2t,
                               d.PV + (size_t)tile * l1 * l2, d.PW + (size_t)tile * l1 * l2);
}

// Only bfloat16-basis variants exist: with a float32 basis the solver forms
// W with the operator kernel and uses the tile kernel (faster there).
hipError_t launch_step(const Desc* d, const int* starts, int count, int total_tiles, int j, int rmax,
                       int basis_bf16, int l1max, int toeplitz, hipStream_t s, int rows) {
    if (!basis_bf16) return hipErrorInvalidValue;
    const int tier = rmax <= 4 ? 4 : (rmax <= 8 ? 8 : 12);
    const bool small = 2 * ((l1max + 15) / 16) <= 8 && rows != 4;
#define RTG_STEP(RR, RPV)                                                                               \
    if (toeplitz)                                                                                       \
        hipLaunchKernelGGL((k_step<RR, RPV, true>), dim3(total_tiles), dim3(256), 0, s, d, starts, count, j); \
    else                                                                                                \
        hipLaunchKernelGGL((k_step<RR, RPV, false>), dim3(total_tiles), dim3(256), 0, s, d, starts, count, j);
#define RTG_STEP_R(RR) if (small) { RTG_STEP(RR, 2) } else { RTG_STEP(RR, 4) }
    if (tier == 4) { RTG_STEP_R(4) } else if (tier == 8) { RTG_STEP_R(8) } else { RTG_STEP_R(12) }
#undef RTG_STEP_R
#undef RTG_STEP
    return hipGetLastError();
}

}  // namespace rtg
