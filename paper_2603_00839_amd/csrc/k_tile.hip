// Fused multi-AXPY, store and mode-wise sketch over one column tile.
//
// A tile is I1 rows x 32 columns (i2) of one channel c, a contiguous block of
// memory in the i1-fastest layout.  Depending on the mode the workgroup
//
//   out = scale * (src - sum_{i<nterms} coef_i V_i)            (multi-AXPY)
//
// which is the orthogonalisation and normalisation of the Arnoldi step
// (Sec. 4.3: W <- W - h_ij V_i, V_{j+1} = W / h_{j+1,j}) or the solution
// update X = X0 + sum_j y_j V_j (Sec. 4.4), stores it, and/or sketches it:
//
//   P[a, b] = sum_{i2 in tile} Om2[b, i2] sum_{i1} Om1[a, i1] out[i1, i2]
//
// (the first two mode products of S(X) = X x_1 Om1 x_2 Om2 x_3 Om3,
// Sec. 3.1).  The mode-1 contraction runs on MFMA directly from the
// registers that hold the tile: with the float32 basis v_mfma_f32_16x16x4f32,
// with the bfloat16 basis v_mfma_f32_16x16x32_bf16 on the stored (rounded)
// values, float32 sources being split into two bfloat16 terms.  Each lane
// owns, for 16 columns, a chunk of RC consecutive rows; since a contraction
// may visit its index in any order, the same chunk serves as the MFMA
// K-slice of both operands.  The four waves split the rows, their partial
// results are summed in LDS, and the mode-2 contraction is a second small
// MFMA product.  The partial P of every tile goes to a buffer that the
// sketched-Gram kernel reduces (and where mode 3 is applied).
#include "rtg_internal.h"

namespace rtg {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

template <int RC>
__device__ __forceinline__ void load_f32(const float* p, float* x) {
#pragma unroll
    for (int q = 0; q < RC; q += 4) {
        f4 v = *gptr((const f4*)(p + q));
        x[q] = v[0]; x[q + 1] = v[1]; x[q + 2] = v[2]; x[q + 3] = v[3];
    }
}

template <int RC>
__device__ __forceinline__ void load_bf16(const bf16_t* p, float* x) {
    if constexpr (RC == 8) {
        u4 v = *gptr((const u4*)p);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            x[2 * q] = __uint_as_float(v[q] << 16);
            x[2 * q + 1] = __uint_as_float(v[q] & 0xffff0000u);
        }
    } else {
        u2 v = *gptr((const u2*)p);
        x[0] = __uint_as_float(v[0] << 16); x[1] = __uint_as_float(v[0] & 0xffff0000u);
        x[2] = __uint_as_float(v[1] << 16); x[3] = __uint_as_float(v[1] & 0xffff0000u);
    }
}

__device__ __forceinline__ bf8 pack_bf8(const bf16_t* h) {
    u4 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (unsigned)h[2 * q] | ((unsigned)h[2 * q + 1] << 16);
    return __builtin_bit_cast(bf8, v);
}

// Om1 fragment (MFMA A operand) of row tile rt for the lane's K-chunk
template <bool BB>
struct AFrag;
template <>
struct AFrag<false> {
    f4 v;
};
template <>
struct AFrag<true> {
    bf8 v;
};

// BB: basis stored as bfloat16 (bf16 MFMA); SRCBF: R0src holds bfloat16;
// RTMAX: row tiles of 16 covering l1 (4 for l1 <= 64, 8 for l1 <= 128).
template <bool BB, bool SRCBF, int RTMAX>
__global__ void __launch_bounds__(256) k_tile(const Desc* __restrict__ descs,
                                              const int* __restrict__ starts, int count,
                                              int mode, int nterms_arg, int dst_index) {
    constexpr int RC = BB ? 8 : 4;          // rows per lane chunk (MFMA K per lane)
    constexpr int KB = 4 * RC;              // rows per K-block (one lane group span)
    constexpr int KPW = BB ? 4 : 8;         // K-blocks per wave in a super-block
    constexpr int SBR = 4 * KPW * KB;       // rows per super-block (4 waves) = 512
    constexpr int TC = TILE_TC;
    constexpr int TCP = TC + 1;

    __shared__ float coef_s[MMAX + 2];
    __shared__ float Ys[LMAX_SPATIAL * TCP];

    const int b = blockIdx.x;
    const int p = find_problem(starts, count, b);
    const Desc& d = descs[p];
    const int tile = b - starts[p];
    if ((mode == TM_SKETCH || mode == TM_NEWV) && d.state[ST_ACTIVE] == 0) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int coll = lane & 15;       // MFMA column (n) / row (m) index
    const int kq = lane >> 4;         // MFMA K-slot group

    const int I1 = d.I1, I2 = d.I2;
    const int l1 = d.l1, l2 = d.l2;
    const int t2 = tile % d.n_i2t, c = tile / d.n_i2t;
    const int i20 = t2 * TC;
    const int ncol = min(TC, I2 - i20);
    const size_t tile_off = (size_t)c * I1 * I2 + (size_t)i20 * I1;
    const size_t es = BB ? 2 : 4;

    int nterms = 0;
    if (mode == TM_NEWV) nterms = nterms_arg;
    else if (mode == TM_ASSEMBLE) nterms = d.state[ST_MEFF];
    const bool do_store = (mode == TM_NEWV || mode == TM_ASSEMBLE);
    const bool do_sketch = (mode != TM_ASSEMBLE);
    const bool src_is_bf = SRCBF && (mode == TM_SKETCH_SRC);

    const void* src;
    if (mode == TM_SKETCH) src = d.W;
    else if (mode == TM_SKETCH_SRC) src = d.R0src;
    else if (mode == TM_NEWV) src = (nterms == 0) ? d.R0src : (const void*)d.W;
    else src = d.X0;     // may be null: zero

    for (int i = tid; i < nterms; i += 256) coef_s[i] = d.coef[i];
    const float scale = do_store ? d.coef[MMAX + 1] : 1.f;
    __syncthreads();

    const int RT = (l1 + 15) >> 4;
    f4 acc[RTMAX][2];
#pragma unroll
    for (int rt = 0; rt < RTMAX; ++rt)
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[rt][g] = f4{0.f, 0.f, 0.f, 0.f};

    // Loads are unconditional from clamped (always in-bounds) addresses and
    // masked afterwards with a select: a branch per load would make the
    // compiler wait for each load before the next one is issued.
    const int nsb = (I1 + SBR - 1) / SBR;
    for (int sb = 0; sb < nsb; ++sb) {
        float x[KPW][2][RC];
        bool ok[KPW][2];
        int offs[KPW][2];             // element offsets from the tile start
        int row0[KPW];
#pragma unroll
        for (int kb = 0; kb < KPW; ++kb) {
            row0[kb] = sb * SBR + (kb * 4 + wave) * KB + RC * kq;
            const int rowc = min(row0[kb], I1 - RC);
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const int col = 16 * g + coll;
                ok[kb][g] = (row0[kb] < I1) && (col < ncol);
                offs[kb][g] = min(col, ncol - 1) * I1 + rowc;
            }
        }
        if (src != nullptr) {
#pragma unroll
            for (int kb = 0; kb < KPW; ++kb)
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    if (src_is_bf) load_bf16<RC>((const bf16_t*)src + tile_off + offs[kb][g], x[kb][g]);
                    else load_f32<RC>((const float*)src + tile_off + offs[kb][g], x[kb][g]);
                }
        } else {
#pragma unroll
            for (int kb = 0; kb < KPW; ++kb)
#pragma unroll
                for (int g = 0; g < 2; ++g)
#pragma unroll
                    for (int q = 0; q < RC; ++q) x[kb][g][q] = 0.f;
        }
        // multi-AXPY over the basis, each term in two halves of K-blocks
        for (int i = 0; i < nterms; ++i) {
            const float ci = coef_s[i];
            const char* vb = (const char*)d.V + ((size_t)i * d.n + tile_off) * es;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float v[KPW / 2][2][RC];
#pragma unroll
                for (int kk = 0; kk < KPW / 2; ++kk)
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        const int kb = h * (KPW / 2) + kk;
                        if (BB) load_bf16<RC>((const bf16_t*)vb + offs[kb][g], v[kk][g]);
                        else load_f32<RC>((const float*)vb + offs[kb][g], v[kk][g]);
                    }
#pragma unroll
                for (int kk = 0; kk < KPW / 2; ++kk)
#pragma unroll
                    for (int g = 0; g < 2; ++g)
#pragma unroll
                        for (int q = 0; q < RC; ++q) {
                            const int kb = h * (KPW / 2) + kk;
                            x[kb][g][q] = fmaf(-ci, v[kk][g][q], x[kb][g][q]);
                        }
            }
        }
#pragma unroll
        for (int kb = 0; kb < KPW; ++kb)
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int q = 0; q < RC; ++q) x[kb][g][q] = ok[kb][g] ? x[kb][g][q] : 0.f;
        // scale, round (bfloat16 basis) and store
        bf16_t h[KPW][2][BB ? RC : 1];
        if (do_store) {
            const bool out_bf = BB && (mode == TM_NEWV);
            char* dstb = (mode == TM_NEWV) ? (char*)d.V + (size_t)dst_index * d.n * es : (char*)d.X;
#pragma unroll
            for (int kb = 0; kb < KPW; ++kb)
#pragma unroll
                for (int g = 0; g < 2; ++g) {
#pragma unroll
                    for (int q = 0; q < RC; ++q) x[kb][g][q] *= scale;
                    if (!ok[kb][g]) continue;
                    const size_t off = tile_off + offs[kb][g];
                    if (out_bf) {
                        if constexpr (BB) {
                            u4 pk;
#pragma unroll
                            for (int q = 0; q < RC; ++q) {
                                h[kb][g][q] = f2bf(x[kb][g][q]);
                                x[kb][g][q] = bf2f(h[kb][g][q]);
                            }
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                pk[q] = (unsigned)h[kb][g][2 * q] | ((unsigned)h[kb][g][2 * q + 1] << 16);
                            *gptr_w((u4*)((bf16_t*)dstb + off)) = pk;
                        }
                    } else {
                        float* o = (float*)dstb + off;
#pragma unroll
                        for (int q = 0; q < RC; q += 4)
                            *gptr_w((f4*)(o + q)) = f4{x[kb][g][q], x[kb][g][q + 1], x[kb][g][q + 2], x[kb][g][q + 3]};
                    }
                }
        }
        if (!do_sketch) continue;
        // mode-1 contraction on MFMA: acc[rt][g] += Om1[16 rt + m, rows] * tile[rows, 16 g + n].
        // The Om1 fragments of the next K-block are loaded while the current
        // one is multiplied.
        auto load_a = [&](int kb, AFrag<BB>* A) {
            const bool rowok = row0[kb] < I1;
            const int rowc = min(row0[kb], I1 - RC);
#pragma unroll
            for (int rt = 0; rt < RTMAX; ++rt) {
                const int a = 16 * rt + coll;
                const bool okA = a < l1 && rowok;
                const size_t off = (size_t)min(a, l1 - 1) * I1 + rowc;
                if constexpr (!BB) {
                    const f4 v = *gptr((const f4*)(d.om1 + off));
                    A[rt].v = okA ? v : f4{0.f, 0.f, 0.f, 0.f};
                } else {
                    const u4 v = *gptr((const u4*)(d.om1h + off));
                    A[rt].v = __builtin_bit_cast(bf8, okA ? v : u4{0u, 0u, 0u, 0u});
                }
            }
        };
        AFrag<BB> Abuf[2][RTMAX];
        load_a(0, Abuf[0]);
#pragma unroll
        for (int kb = 0; kb < KPW; ++kb) {
            AFrag<BB>* A = Abuf[kb & 1];
            if (kb + 1 < KPW) load_a(kb + 1, Abuf[(kb + 1) & 1]);
            if constexpr (!BB) {
                f4 B[2];
#pragma unroll
                for (int g = 0; g < 2; ++g)
                    B[g] = f4{x[kb][g][0], x[kb][g][1], x[kb][g][2], x[kb][g][3]};
#pragma unroll
                for (int rt = 0; rt < RTMAX; ++rt) {
                    if (rt >= RT) break;
#pragma unroll
                    for (int g = 0; g < 2; ++g)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc[rt][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[rt].v[q], B[g][q], acc[rt][g], 0, 0, 0);
                }
            } else {
                // bfloat16 operands: exact for a bfloat16 tile, hi + lo split for float32
                const bool split = !(mode == TM_NEWV || src_is_bf);
                bf8 Bh[2], Bl[2];
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    bf16_t hi[8], lo[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        hi[q] = f2bf(x[kb][g][q]);
                        lo[q] = split ? f2bf(x[kb][g][q] - bf2f(hi[q])) : (bf16_t)0;
                    }
                    Bh[g] = pack_bf8(hi);
                    Bl[g] = pack_bf8(lo);
                }
#pragma unroll
                for (int rt = 0; rt < RTMAX; ++rt) {
                    if (rt >= RT) break;
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        acc[rt][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[rt].v, Bh[g], acc[rt][g], 0, 0, 0);
                        if (split)
                            acc[rt][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[rt].v, Bl[g], acc[rt][g], 0, 0, 0);
                    }
                }
            }
        }
    }
    if (!do_sketch) return;

    // ---- sum the four waves' mode-1 partials: Ys[a][col] (deterministic order)
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int rt = 0; rt < RTMAX; ++rt) {
                if (rt >= RT) break;
#pragma unroll
                for (int g = 0; g < 2; ++g)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int a = 16 * rt + 4 * kq + i;
                        const int col = 16 * g + coll;
                        float v = acc[rt][g][i];
                        if (w > 0) v += Ys[a * TCP + col];
                        Ys[a * TCP + col] = v;
                    }
            }
        }
        __syncthreads();
    }
    // ---- mode-2 contraction: P[a][b] = sum_k Ys[a][k] Om2[b][i20 + k]
    const int RT2 = (l2 + 15) >> 4;
    float* P = ((mode == TM_NEWV) ? d.PV : d.PW) + (size_t)tile * l1 * l2;
    for (int t = wave; t < RT * RT2; t += 4) {
        const int rt = t / RT2, rt2 = t % RT2;
        f4 pacc = f4{0.f, 0.f, 0.f, 0.f};
        const int a = 16 * rt + coll;
        const int bcol = 16 * rt2 + coll;
        // rows a >= l1 of Ys hold zeros; Om2 loads are clamped and masked
        float Bv[TC / 4];
#pragma unroll
        for (int ks = 0; ks < TC / 4; ++ks) {
            const int k = 4 * ks + kq;
            const float v = *gptr(d.om2 + (size_t)min(bcol, l2 - 1) * I2 + i20 + min(k, ncol - 1));
            Bv[ks] = (bcol < l2 && k < ncol) ? v : 0.f;
        }
#pragma unroll
        for (int ks = 0; ks < TC / 4; ++ks) {
            const int k = 4 * ks + kq;
            pacc = __builtin_amdgcn_mfma_f32_16x16x4f32(Ys[a * TCP + k], Bv[ks], pacc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ar = 16 * rt + 4 * kq + i;
            if (ar < l1 && bcol < l2) *gptr_w(P + (size_t)ar * l2 + bcol) = pacc[i];
        }
    }
}

hipError_t launch_tile(const Desc* d, const int* starts, int count, int total_tiles, int mode,
                       int nterms, int dst_index, int basis_bf16, int src_bf16, int l1max, hipStream_t s) {
#define RTG_TILE(BBV, SBV, RTV)                                                                  \
    hipLaunchKernelGGL((k_tile<BBV, SBV, RTV>), dim3(total_tiles), dim3(256), 0, s, d, starts, count, \
                       mode, nterms, dst_index)
    const bool small = l1max <= 64;
    if (basis_bf16) {
        if (src_bf16) { if (small) RTG_TILE(true, true, 4); else RTG_TILE(true, true, 8); }
        else { if (small) RTG_TILE(true, false, 4); else RTG_TILE(true, false, 8); }
    } else {
        if (small) RTG_TILE(false, false, 4); else RTG_TILE(false, false, 8);
    }
#undef RTG_TILE
    return hipGetLastError();
}

}  // namespace rtg
