#pragma once
// Fused multi-AXPY, store and mode-wise sketches over one column tile.
//
// A tile is I1 rows x 32 columns (i2) of one channel c, a contiguous block of
// memory in the i1-fastest layout.  Depending on the mode the workgroup
//
//   out = scale * (src - sum_{i<nterms} coef_i V_i)            (multi-AXPY)
//
// which is the orthogonalisation and normalisation of the Arnoldi step
// (Sec. 4.3: W <- W - h_ij V_i, V_{j+1} = W / h_{j+1,j}), a Golub-Kahan
// half-step (Sec. 4.5: one term, U_{k+1} = (Phi(V_k) - alpha_k U_k) / beta_{k+1}
// or V_{k+1} = (Phi^T(U_{k+1}) - beta_{k+1} V_k) / alpha_{k+1}, where the
// composed matrices belong to the operator of the side written) or the
// solution update X = X0 + sum_j y_j V_j (Sec. 4.4), stores it, and/or
// sketches it:
//
//   P[a, b] = sum_{i2 in tile} Om2[b, i2] sum_{i1} Om1[a, i1] out[i1, i2]
//
// (the first two mode products of S(X) = X x_1 Om1 x_2 Om2 x_3 Om3,
// Sec. 3.1).  A new basis tensor is sketched twice in the same pass: with
// (Om1, Om2) for S(V_{j+1}) and with the composed matrices (Om1 A1, Om2 A2)
// for S(Phi(V_{j+1})), because mode products compose and Phi is the mode-wise
// product with (A1, A2, B^T) (eq. (2)).  The next step's sketched inner
// products then need no separate pass over W = Phi(V_{j+1}).
//
// Phase 1 (per super-block of 256 rows): every lane owns 32 elements of the
// tile, accumulates the multi-AXPY in float32 registers, stores the result
// (rounded to bfloat16 for a bfloat16 basis) and writes it to LDS, column-
// major.  Phase 2: the four waves split the (stacked) sketch rows and run the
// mode-1 contraction on MFMA with the tile from LDS as the B operand
// (v_mfma_f32_16x16x4f32 for a float32 basis, v_mfma_f32_16x16x32_bf16 for a
// bfloat16 one; a float32 tile in bfloat16 mode is split into high and low
// bfloat16 planes, and so is the composed matrix Om1 A1).  After the last
// super-block the mode-2 contraction is a second small MFMA product, and the
// partial P of every tile goes to a buffer that the sketched-Gram kernel
// reduces (applying mode 3).

#include "rtg_internal.h"

namespace rtg {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

constexpr int TILE_SBR = 256;   // rows per super-block: 256 lanes x 32 elements / 32 columns
// element offset of a chunk outside the tile: its byte offset lies past every
// buffer extent used here (a tile spans 32 x I1 elements of at most 4 bytes)
constexpr unsigned OOB_ELEM = 0x20000000u;
// byte offset past the operand-order sketch matrices (under 1 GiB a plane)
constexpr unsigned OOB_A = 0x80000000u;

// raw buffer resource over [base, base + bytes): loads past the end return
// zero and stores past it are dropped
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

template <bool MB, bool SPLIT, int RPW>
struct TileSmem {
    static constexpr int TC = TILE_TC;
    static constexpr int CSB = TILE_SBR + 8;    // bfloat16 plane column stride (elements)
    static constexpr int CSF = TILE_SBR + 4;    // float32 column stride (elements)
    static constexpr int XBYTES = MB ? (SPLIT ? 2 : 1) * TC * CSB * 2 : TC * CSF * 4;
    static constexpr int YP = TC + 1;
    static constexpr int YBYTES = 64 * RPW * YP * 4;   // stacked sketch rows x columns
    static constexpr int BYTES = XBYTES > YBYTES ? XBYTES : YBYTES;
};

// LDS of one tile workgroup
template <bool MB, bool SPLIT, int RPW>
struct TileShared {
    float coef_s[MMAX + 2];
    __attribute__((aligned(16))) unsigned char smem[TileSmem<MB, SPLIT, RPW>::BYTES];
};

// BB: basis stored as bfloat16; MB: the sketch contractions take bfloat16
// MFMA operands (float32 accumulation) -- a bfloat16 basis always does, a
// float32 basis in the mixed form (RTG_F32_BF16) does with its tile rounded
// to bfloat16 for the products; SPLIT: the sketched tile is float32 in
// bfloat16 mode, split into two planes; RPW: sketch row tiles of 16 per wave.
template <bool BB, bool MB, bool SPLIT, int RPW>
__device__ __forceinline__ void tile_task(const Desc* __restrict__ descs, const int* __restrict__ starts,
                                          int count, int mode, int nterms_arg, int dst_index, int t0, int b,
                                          TileShared<MB, SPLIT, RPW>& sh) {
    static_assert(MB || !BB, "a bfloat16 basis uses bfloat16 products");
    using SM = TileSmem<MB, SPLIT, RPW>;
    constexpr int TC = TILE_TC;
    constexpr int SBR = TILE_SBR;
    constexpr int CK = BB ? 8 : 4;             // elements per lane chunk (16 bytes of basis)
    constexpr int NCK = SBR * TC / 256 / CK;   // chunks per lane
    constexpr int KBR = MB ? 32 : 16;          // rows per MFMA K-block
    constexpr int CSB = SM::CSB, CSF = SM::CSF, YP = SM::YP;

    float* coef_s = sh.coef_s;
    unsigned char* smem = sh.smem;
    bf16_t* Xh = (bf16_t*)smem;                 // high (or only) bfloat16 plane
    bf16_t* Xl = Xh + TC * CSB;                 // low plane (SPLIT)
    float* Xf = (float*)smem;                   // float32 tile
    float* Ys = (float*)smem;                   // mode-1 results (after the last super-block)

    const int p = find_problem(starts, count, b);
    const Desc& d = descs[p];
    const int tile = uniform_int(b - starts[p]);
    const bool newv = (mode == TM_NEWV || mode == TM_GKNEW || mode == TM_NEWV1);
    // V_1 stored by the operator kernel already: sketched from the basis
    const bool v1_stored = (mode == TM_NEWV1) && d.X0 != nullptr;
    if ((newv || mode == TM_SKETCH_W) && d.state[ST_ACTIVE] == 0) return;
    if (mode == TM_ASSEMBLE && d.state[ST_SKIP] != 0) return;   // X stays (restart cycle sat out)

    const int tid = block_tid();
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m16 = lane & 15;        // MFMA row (A) / column (B) index
    const int kq = lane >> 4;         // MFMA K group

    const int I1 = d.I1, I2 = d.I2;
    const int l1 = d.l1, l2 = d.l2;
    const int t2 = tile % d.n_i2t, c = tile / d.n_i2t;
    const int i20 = t2 * TC;
    const int ncol = min(TC, I2 - i20);
    const size_t tile_off = (size_t)c * I1 * I2 + (size_t)i20 * I1;
    const size_t es = BB ? 2 : 4;

    int nterms = 0;
    if (newv) nterms = nterms_arg;
    else if (mode == TM_ASSEMBLE) nterms = uniform_int(d.state[ST_MEFF]);
    const int first = (mode == TM_GKNEW) ? t0 : 0;   // terms [first, nterms)
    const bool do_store = (newv || mode == TM_ASSEMBLE) && !v1_stored;
    const bool do_sketch = (mode != TM_ASSEMBLE) && !d.unsketched;   // an identity sketch keeps no partials
    const bool dual = newv && d.st == nullptr;   // a general PSF has no composed sketch matrices
    const bool src_is_bf = BB && !SPLIT && (mode == TM_SKETCH_SRC || v1_stored);

    const void* src;
    if (mode == TM_SKETCH_SRC) src = d.R0src;
    else if (mode == TM_SKETCH_W) src = d.W;
    else if (mode == TM_NEWV) src = (nterms == 0) ? d.R0src : (const void*)d.W;
    else if (mode == TM_NEWV1) src = v1_stored ? (const void*)d.V : d.R0src;
    else if (mode == TM_GKNEW) src = d.W;
    else src = d.X0;     // may be null: zero
    src = uniform_ptr(src);

    for (int i = tid; i < nterms; i += 256) coef_s[i] = d.coef[i];
    const float scale = do_store ? d.coef[MMAX + 1] : 1.f;
    __syncthreads();

    const int RT = (l1 + 15) >> 4;
    const int NRT = dual ? 2 * RT : RT;       // stacked row tiles: [Om1 ; Om1 A1]
    // sketch matrices in operand order: Om1, and Om1 A1 (bfloat16: high
    // plane then low plane)
    const int nkbf = frag_nkb(I1, KBR);
    const unsigned fbytes = (unsigned)frag_elems(l1, I1, KBR) * (MB ? 2u : 4u);
    const auto rom1 = make_rsrc(MB ? (const void*)d.om1hf : (const void*)d.om1f, (int)fbytes);
    const auto rom1c = make_rsrc(MB ? (const void*)d.om1th : (const void*)d.om1t, (int)(MB ? 2 * fbytes : fbytes));
    f4 acc[RPW][2];
#pragma unroll
    for (int u = 0; u < RPW; ++u)
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[u][g] = f4{0.f, 0.f, 0.f, 0.f};

    // chunk u of this lane: column col[u], rows row[u] .. row[u] + CK - 1 of the super-block
    int colu[NCK], rowu[NCK];
#pragma unroll
    for (int u = 0; u < NCK; ++u) {
        const int e = (u * 256 + tid) * CK;
        colu[u] = e / SBR;
        rowu[u] = e % SBR;
    }

    const int nsb = (I1 + SBR - 1) / SBR;
    for (int sb = 0; sb < nsb; ++sb) {
        // ---- phase 1: multi-AXPY, store, LDS.  Loads are unconditional from
        // clamped (always in-bounds) addresses and masked afterwards, so that
        // they stay in flight together.
        // Buffer loads and stores with per-lane byte offsets from a uniform
        // base: a chunk outside the tile gets an offset past the buffer's
        // extent, so the hardware returns zeros for its loads and drops its
        // stores -- no branches, no clamping, all loads in flight together.
        unsigned offs[NCK];
#pragma unroll
        for (int u = 0; u < NCK; ++u) {
            const int rg = sb * SBR + rowu[u];
            offs[u] = ((rg < I1) & (colu[u] < ncol)) ? (unsigned)(colu[u] * I1 + rg) : OOB_ELEM;
        }
        const int tile_elems = ncol * I1;
        float x[NCK][CK];
        if (src == nullptr) {
#pragma unroll
            for (int u = 0; u < NCK; ++u)
#pragma unroll
                for (int q = 0; q < CK; ++q) x[u][q] = 0.f;
        } else if (src_is_bf) {
            const auto rs = make_rsrc((const char*)src + tile_off * 2, tile_elems * 2);
#pragma unroll
            for (int u = 0; u < NCK; ++u) {
                const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, offs[u] * 2u, 0, 0);
#pragma unroll
                for (int q = 0; q < CK / 2; ++q) {
                    x[u][2 * q] = __uint_as_float(v[q] << 16);
                    x[u][2 * q + 1] = __uint_as_float(v[q] & 0xffff0000u);
                }
            }
        } else {
            const auto rs = make_rsrc((const char*)src + tile_off * 4, tile_elems * 4);
#pragma unroll
            for (int u = 0; u < NCK; ++u)
#pragma unroll
                for (int q = 0; q < CK; q += 4) {
                    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, offs[u] * 4u + q * 4u, 0, 0);
                    x[u][q] = __uint_as_float(v[0]); x[u][q + 1] = __uint_as_float(v[1]);
                    x[u][q + 2] = __uint_as_float(v[2]); x[u][q + 3] = __uint_as_float(v[3]);
                }
        }
        // multi-AXPY, software-pipelined: the next stage's loads are in
        // flight while the current stage is applied.  A stage is one term
        // (bfloat16 basis: 4 chunks) or half a term (float32: 4 of 8 chunks).
        constexpr int SPT = BB ? 1 : 2;          // stages per term
        constexpr int CPS = NCK / SPT;           // chunks per stage
        const int nst = (nterms - first) * SPT;
        auto load_stage = [&](int st, u4* v) {
            const int i = first + st / SPT, c0 = (st % SPT) * CPS;
            const auto rv = make_rsrc((const char*)d.V + ((size_t)i * d.n + tile_off) * es, tile_elems * (int)es);
#pragma unroll
            for (int u = 0; u < CPS; ++u)
                v[u] = __builtin_amdgcn_raw_buffer_load_b128(rv, offs[c0 + u] * (unsigned)es, 0, 0);
        };
        auto apply_stage = [&](int st, const u4* v) {
            const float ci = coef_s[first + st / SPT];
            const int c0 = (st % SPT) * CPS;
#pragma unroll
            for (int uu = 0; uu < CPS; ++uu)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if constexpr (BB) {
                        x[uu][2 * q] = fmaf(-ci, __uint_as_float(v[uu][q] << 16), x[uu][2 * q]);
                        x[uu][2 * q + 1] = fmaf(-ci, __uint_as_float(v[uu][q] & 0xffff0000u), x[uu][2 * q + 1]);
                    } else {
                        // c0 is 0 or CPS: select the half with a uniform branch-free index
                        float& xr = (c0 == 0) ? x[uu][q] : x[CPS + uu][q];
                        xr = fmaf(-ci, __uint_as_float(v[uu][q]), xr);
                    }
                }
        };
        u4 va[CPS], vb[CPS];
        if (nst > 0) load_stage(0, va);
        for (int st = 0; st < nst; st += 2) {
            if (st + 1 < nst) load_stage(st + 1, vb);
            apply_stage(st, va);
            if (st + 1 < nst) {
                if (st + 2 < nst) load_stage(st + 2, va);
                apply_stage(st + 1, vb);
            }
        }
        // scale (chunks outside the tile are zero already), round (bfloat16 basis), store
#pragma unroll
        for (int u = 0; u < NCK; ++u)
#pragma unroll
            for (int q = 0; q < CK; ++q) x[u][q] *= scale;
        if (newv && BB && do_store) {
            const auto rd = make_rsrc((const char*)d.V + ((size_t)dst_index * d.n + tile_off) * 2, tile_elems * 2);
#pragma unroll
            for (int u = 0; u < NCK; ++u) {
                u4 pk;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    pk[q] = (unsigned)f2bf(x[u][2 * q]) | ((unsigned)f2bf(x[u][2 * q + 1]) << 16);
                __builtin_amdgcn_raw_buffer_store_b128(pk, rd, offs[u] * 2u, 0, 0);
            }
        } else if (do_store) {
            const char* db = newv ? (const char*)d.V + ((size_t)dst_index * d.n + tile_off) * 4
                                               : (const char*)d.X + tile_off * 4;
            const auto rd = make_rsrc(db, tile_elems * 4);
#pragma unroll
            for (int u = 0; u < NCK; ++u)
#pragma unroll
                for (int q = 0; q < CK; q += 4) {
                    const u4 pk = u4{__float_as_uint(x[u][q]), __float_as_uint(x[u][q + 1]),
                                     __float_as_uint(x[u][q + 2]), __float_as_uint(x[u][q + 3])};
                    __builtin_amdgcn_raw_buffer_store_b128(pk, rd, offs[u] * 4u + q * 4u, 0, 0);
                }
        }
        if (!do_sketch) continue;
        if (sb > 0) __syncthreads();          // the previous super-block's MFMA reads are done
#pragma unroll
        for (int u = 0; u < NCK; ++u) {
            if constexpr (MB && !BB && !SPLIT) {
                // float32 basis, bfloat16 products: the chunk's four values rounded
                u2v hi;
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    hi[q] = (unsigned)f2bf(x[u][2 * q]) | ((unsigned)f2bf(x[u][2 * q + 1]) << 16);
                *(u2v*)(Xh + colu[u] * CSB + rowu[u]) = hi;
            } else if constexpr (MB && !BB) {
                // float32 source split into high and low planes
                u2v hi, lo;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const bf16_t h0 = f2bf(x[u][2 * q]), h1 = f2bf(x[u][2 * q + 1]);
                    hi[q] = (unsigned)h0 | ((unsigned)h1 << 16);
                    const bf16_t g0 = f2bf(x[u][2 * q] - bf2f(h0)), g1 = f2bf(x[u][2 * q + 1] - bf2f(h1));
                    lo[q] = (unsigned)g0 | ((unsigned)g1 << 16);
                }
                *(u2v*)(Xh + colu[u] * CSB + rowu[u]) = hi;
                *(u2v*)(Xl + colu[u] * CSB + rowu[u]) = lo;
            } else if constexpr (BB) {
                u4 hi, lo;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bf16_t h0 = f2bf(x[u][2 * q]), h1 = f2bf(x[u][2 * q + 1]);
                    hi[q] = (unsigned)h0 | ((unsigned)h1 << 16);
                    if constexpr (SPLIT) {
                        const bf16_t g0 = f2bf(x[u][2 * q] - bf2f(h0)), g1 = f2bf(x[u][2 * q + 1] - bf2f(h1));
                        lo[q] = (unsigned)g0 | ((unsigned)g1 << 16);
                    }
                }
                *(u4*)(Xh + colu[u] * CSB + rowu[u]) = hi;
                if constexpr (SPLIT) *(u4*)(Xl + colu[u] * CSB + rowu[u]) = lo;
            } else {
                *(f4*)(Xf + colu[u] * CSF + rowu[u]) = f4{x[u][0], x[u][1], x[u][2], x[u][3]};
            }
        }
        __syncthreads();

        // ---- phase 2: mode-1 contraction of this super-block on MFMA.
        // Wave w owns stacked row tiles w, w + 4, ...; rows of tile t are
        // rows of Om1 (t < RT) or of Om1 A1 (RT <= t < 2 RT).
        const int rows_sb = min(SBR, I1 - sb * SBR);
        const int nkb = (rows_sb + KBR - 1) / KBR;
        struct AF {
            u4 h, l;     // bfloat16 products: Om1 (h), or Om1 A1 high / low; float32: h as f4 bits
        };
        // A fragments in operand order: one contiguous 1 KB read per wave and
        // tile; padding rows and columns are stored zeros, and unused tiles
        // (t >= NRT) read nothing (offset past the buffer range)
        auto load_a = [&](int kb, AF* A) {
            const int kbg = sb * (SBR / KBR) + kb;
#pragma unroll
            for (int u = 0; u < RPW; ++u) {
                const int t = wave + 4 * u;
                const bool half = t >= RT;
                const int tl = t - (half ? RT : 0);
                const unsigned off = (t < NRT) ? (unsigned)((tl * nkbf + kbg) * 64 + lane) * 16u : OOB_A;
                const auto& rs = half ? rom1c : rom1;
                A[u].h = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
                if constexpr (MB)
                    A[u].l = half ? __builtin_amdgcn_raw_buffer_load_b128(rs, off + fbytes, 0, 0) : u4{0u, 0u, 0u, 0u};
            }
        };
        auto mfma_block = [&](int kb, const AF* A) {
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const int col = 16 * g + m16;
                if constexpr (MB) {
                    const u4 bh = *(const u4*)(Xh + col * CSB + kb * KBR + 8 * kq);
                    u4 bl = u4{0u, 0u, 0u, 0u};
                    if constexpr (SPLIT) bl = *(const u4*)(Xl + col * CSB + kb * KBR + 8 * kq);
#pragma unroll
                    for (int u = 0; u < RPW; ++u) {
                        const int t = wave + 4 * u;
                        if (t >= NRT) break;
                        acc[u][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf8, A[u].h), __builtin_bit_cast(bf8, bh), acc[u][g], 0, 0, 0);
                        if (t >= RT)
                            acc[u][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf8, A[u].l), __builtin_bit_cast(bf8, bh), acc[u][g], 0, 0, 0);
                        if constexpr (SPLIT)
                            acc[u][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf8, A[u].h), __builtin_bit_cast(bf8, bl), acc[u][g], 0, 0, 0);
                    }
                } else {
                    const f4 bv = *(const f4*)(Xf + col * CSF + kb * KBR + 4 * kq);
#pragma unroll
                    for (int u = 0; u < RPW; ++u) {
                        const int t = wave + 4 * u;
                        if (t >= NRT) break;
                        const f4 av = __builtin_bit_cast(f4, A[u].h);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc[u][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv[q], acc[u][g], 0, 0, 0);
                    }
                }
            }
        };
        // the fragments of the next K-block are loaded while the current one
        // is multiplied (two named buffers: no dynamically indexed arrays)
        AF A0[RPW], A1[RPW];
        load_a(0, A0);
        for (int kb = 0; kb < nkb; kb += 2) {
            if (kb + 1 < nkb) load_a(kb + 1, A1);
            mfma_block(kb, A0);
            if (kb + 1 < nkb) {
                if (kb + 2 < nkb) load_a(kb + 2, A0);
                mfma_block(kb + 1, A1);
            }
        }
    }
    if (!do_sketch) return;

    // ---- mode-1 results to LDS: Ys[16 t + r][col]
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
        const int t = wave + 4 * u;
        if (t >= NRT) break;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) Ys[(16 * t + 4 * kq + i) * YP + 16 * g + m16] = acc[u][g][i];
    }
    __syncthreads();

    // ---- mode-2 contraction: P[a][b] = sum_k Ys[a][k] Om2x[b][i20 + k]
    float* Pt0 = (newv ? d.PV : d.PW) + (size_t)tile * l1 * l2;
    float* Pt1 = d.PW + (size_t)tile * l1 * l2;
    mode2_partials<TC, YP>(Ys, wave, lane, NRT, RT, l1, l2, I2, i20, ncol, d.om2, d.om2t, Pt0, Pt1);
}

}  // namespace rtg
