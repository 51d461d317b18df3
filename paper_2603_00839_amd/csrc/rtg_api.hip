// C ABI of librtg.so (declared in include/rtg.h): handles, workspace layout,
// argument checks and the launch sequence of an RTG-GMRES solve
// (algorithm "Block GMRES via Sketched Einstein Product", Sec. 4.4, with the
// sketched global Arnoldi process of Sec. 4.3).
//
// Per problem the sequence is
//   Om1 A1, Om2 A2, Om3 B^T                k_compose (sketch of Phi(X) as a sketch of X)
//   R0 = C - Phi(X0)                       k_phi   (skipped when X0 = 0)
//   partial sketches of R0                 k_tile  (sketch)
//   beta = ||S(R0)||                       k_gram  (start)
//   V1 = R0 / beta, partial S(V1), S(Phi(V1))                       k_tile
//   for j = 1..m:
//     S(V_j), S(Phi(V_j)), h_{:,j}, h_{j+1,j}, Givens               k_gram  (step)
//     V_{j+1} = (Phi(V_j) - sum h_ij V_i) / h_{j+1,j},
//     partial S(V_{j+1}), S(Phi(V_{j+1})):
//       bfloat16 basis: Phi(V_j) formed tile by tile       k_step
//       float32 basis:  W = Phi(V_j)                      k_phi, then k_tile
//   projected Tikhonov problem, mu         k_solve
//   X = X0 + sum y_j V_j                   k_tile  (assemble)
// Every launch covers all problems of a batch; the host never waits.
#include "rtg_internal.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <vector>

struct rtg_op_s {
    int I1, I2, J, r1, r2, rB;
    float* a1;
    float* a2;
    float* bb;
    float* a1t;   // transposed bands: a1t[(r1 + dd) I1 + i] = a1[i (2 r1 + 1) + r1 + dd]
    float* a2t;
    float* a1p[3];  // A1 band rows zero-padded to the operator tiers R = 4, 8, 12:
                    // a1p[k][i * WP + R + dd] = A1[i, i + dd], WP = 2R + 1 rounded up to 4
    int toeplitz;   // A1 and A2 are Toeplitz on their in-range entries (convolutions with zero BC)
    float* taps;    // their taps: taps[r1 + dd] = A1[i, i + dd], then RMAX_SPATIAL * 2 + 1 on, A2's
    rtg_op_s* adj;  // the adjoint Phi^T(X) = X x_1 A1^T x_2 A2^T x_3 B (transposed bands), for Golub-Kahan
    float* st;      // general PSF (rtg_setup_operator_psf): stencil st[(a + r) (2r + 1) + b + r], the weight of
                    // X[i1 + a, i2 + b] (the PSF rotated by 180 degrees); r1 = r2 = r, no bands
};

struct rtg_sk_s {
    int I1, I2, J, l1, l2, l3, has_om3;
    float* om1;
    float* om2;
    float* om3;
    rtg::bf16_t* om1h;
    float* om1f;          // Om1 in MFMA operand order (float32 tiles)
    rtg::bf16_t* om1hf;   // bfloat16 Om1 in MFMA operand order
    int identity;         // all three factors the identity: unsketched inner products
};

namespace {

using namespace rtg;

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

struct Layout {
    size_t V, W, PW, PV, SV, dots, G, H, R, gv, coef, y, state, scal, ot1, ot1h, ot2, ot3, total;
    int n_i2t, ntile_tile, ntile_gram, ntile_phi;
};

Layout problem_layout(const rtg_op_s* op, const rtg_sk_s* sk, int m, int bf16) {
    Layout L{};
    const size_t n = (size_t)op->I1 * op->I2 * op->J;
    const size_t Ls = (size_t)sk->l1 * sk->l2 * sk->l3;
    const size_t es = bf16 ? 2 : 4;
    L.n_i2t = (op->I2 + TILE_TC - 1) / TILE_TC;
    L.ntile_tile = op->J * L.n_i2t;
    const int ch = gram_pairs_per_block(sk->l3, op->J, L.n_i2t);
    L.ntile_gram = sk->identity ? frob_wgs((long long)n) : (sk->l1 * sk->l2 + ch - 1) / ch;
    L.ntile_phi = phi_tiles(op->I1, op->I2, op->J, phi_jt(op->J));
    // an identity sketch keeps no partials, stored sketches or composed matrices
    const bool sk_bufs = !sk->identity;
    const size_t part = sk_bufs ? (size_t)L.ntile_tile * sk->l1 * sk->l2 * sizeof(float) : 0;
    size_t off = 0;
    auto take = [&](size_t bytes) { off = align_up(off); size_t at = off; off += bytes; return at; };
    L.V = take((size_t)(m + 1) * n * es);
    L.W = take(n * sizeof(float));
    L.PW = take(part);
    L.PV = take(part);
    L.SV = take(sk_bufs ? (size_t)(m + 1) * Ls * sizeof(float) : 0);
    L.dots = take((size_t)L.ntile_gram * (MMAX + 2) * 2 * sizeof(double));
    L.G = take((size_t)(m + 1) * (m + 1) * sizeof(double));
    L.H = take((size_t)(m + 1) * m * sizeof(double));
    L.R = take((size_t)m * m * sizeof(double));
    L.gv = take((size_t)(3 * m + 1) * sizeof(double));
    L.coef = take((MMAX + 2) * sizeof(float));
    L.y = take((size_t)m * sizeof(double));
    L.state = take(NSTATE * sizeof(int));
    L.scal = take(NSCAL * sizeof(double));
    L.ot1 = take(sk_bufs ? frag_elems(sk->l1, op->I1, FRAG_K_F32) * sizeof(float) : 0);
    L.ot1h = take(sk_bufs ? 2 * frag_elems(sk->l1, op->I1, FRAG_K_BF16) * sizeof(bf16_t) : 0);
    L.ot2 = take(sk_bufs ? (size_t)sk->l2 * op->I2 * sizeof(float) : 0);
    L.ot3 = take(sk_bufs ? (size_t)sk->l3 * op->J * sizeof(float) : 0);
    L.total = align_up(off);
    return L;
}

// Golub-Kahan keeps a second basis (U_1..U_{m+1}), its stored sketches and
// the composed sketch matrices of Phi^T after the layout above; everything
// else (W, the partials, the bidiagonal matrix in H, rotations, state) is
// shared by the two sides, which never run at the same time.
struct GKExtra {
    size_t V, SV, ot1, ot1h, ot2, ot3, total;
};

GKExtra gk_extra_layout(const rtg_op_s* op, const rtg_sk_s* sk, int m, int bf16) {
    GKExtra E{};
    const size_t n = (size_t)op->I1 * op->I2 * op->J;
    const size_t Ls = (size_t)sk->l1 * sk->l2 * sk->l3;
    size_t off = 0;
    auto take = [&](size_t bytes) { off = align_up(off); size_t at = off; off += bytes; return at; };
    E.V = take((size_t)(m + 1) * n * (bf16 ? 2 : 4));
    E.SV = take((size_t)(m + 1) * Ls * sizeof(float));
    E.ot1 = take(frag_elems(sk->l1, op->I1, FRAG_K_F32) * sizeof(float));
    E.ot1h = take(2 * frag_elems(sk->l1, op->I1, FRAG_K_BF16) * sizeof(bf16_t));
    E.ot2 = take((size_t)sk->l2 * op->I2 * sizeof(float));
    E.ot3 = take((size_t)sk->l3 * op->J * sizeof(float));
    E.total = align_up(off);
    return E;
}

// The U side of a Golub-Kahan problem from its filled V side d: operator
// Phi^T, its own basis, stored sketches and composed matrices at ub; the
// rest of the workspace is shared.
void fill_gk_sides(Desc& d, Desc& u, const rtg_op_s* op, const rtg_sk_s* sk, int m, int bf16, char* ub) {
    const GKExtra E = gk_extra_layout(op, sk, m, bf16);
    u = d;
    const rtg_op_s* a = op->adj;
    u.a1 = a->a1; u.a2 = a->a2; u.bb = a->bb;
    u.a1t = a->a1t; u.a2t = a->a2t;
    for (int k = 0; k < 3; ++k) u.a1p[k] = a->a1p[k];
    u.toeplitz = a->toeplitz;
    u.taps = a->taps;
    u.V = ub + E.V;
    u.SV = (float*)(ub + E.SV);
    u.om1t = (const float*)(ub + E.ot1);
    u.om1th = (const bf16_t*)(ub + E.ot1h);
    u.om2t = (const float*)(ub + E.ot2);
    u.om3t = (const float*)(ub + E.ot3);
    d.gk = 1;
    u.gk = 2;
    d.SVx = u.SV;
    u.SVx = d.SV;
}

size_t problem_bytes(const rtg_op_s* op, const rtg_sk_s* sk, int m, int bf16, int method) {
    size_t b = problem_layout(op, sk, m, bf16).total;
    if (method == RTG_METHOD_GOLUB_KAHAN) b += gk_extra_layout(op, sk, m, bf16).total;
    return b;
}

// descriptors (nsides per problem: Golub-Kahan has a V side and a U side;
// restarted solves keep a second copy for the restart cycles) and the
// per-kernel tile prefix tables
size_t plan_bytes(int count, int nsides = 1, bool restart = false) {
    return align_up((size_t)count * nsides * (restart ? 2 : 1) * sizeof(Desc)) +
           align_up((size_t)NKIND * (count + 1) * sizeof(int)) + align_up(SCH_WORDS * sizeof(int));
}

int check_pair(const rtg_op_s* op, const rtg_sk_s* sk) {
    if (!op || !sk) return RTG_E_ARG;
    if (op->I1 != sk->I1 || op->I2 != sk->I2 || op->J != sk->J) return RTG_E_SHAPE;
    return RTG_OK;
}

int check_m(const rtg_sk_s* sk, int m) {
    const long long L = (long long)sk->l1 * sk->l2 * sk->l3;
    if (m < 1 || m > MMAX || m + 1 > L) return RTG_E_SHAPE;
    return RTG_OK;
}

void fill_desc(Desc& d, const rtg_op_s* op, const rtg_sk_s* sk, int m, int bf16, char* base,
               const Layout& L) {
    std::memset(&d, 0, sizeof(d));
    d.I1 = op->I1; d.I2 = op->I2; d.J = op->J;
    d.l1 = sk->l1; d.l2 = sk->l2; d.l3 = sk->l3;
    d.r1 = op->r1; d.r2 = op->r2; d.rB = op->rB;
    d.m = m;
    d.bf16 = bf16;
    d.skbf = bf16;
    d.has_om3 = sk->has_om3;
    d.n_i2t = L.n_i2t;
    d.ntile[KIND_PHI] = L.ntile_phi;
    d.ntile[KIND_TILE] = L.ntile_tile;
    d.ntile[KIND_GRAM] = L.ntile_gram;
    d.n = (long long)op->I1 * op->I2 * op->J;
    d.L = (long long)sk->l1 * sk->l2 * sk->l3;
    d.a1 = op->a1; d.a2 = op->a2; d.bb = op->bb;
    d.a1t = op->a1t; d.a2t = op->a2t;
    for (int k = 0; k < 3; ++k) d.a1p[k] = op->a1p[k];
    d.toeplitz = op->toeplitz;
    d.taps = op->taps;
    d.st = op->st;
    d.unsketched = sk->identity;
    d.om1 = sk->om1; d.om1h = sk->om1h; d.om2 = sk->om2; d.om3 = sk->om3;
    d.om1f = sk->om1f; d.om1hf = sk->om1hf;
    if (base) {
        d.V = base + L.V;
        d.W = (float*)(base + L.W);
        d.PW = (float*)(base + L.PW);
        d.PV = (float*)(base + L.PV);
        d.SV = (float*)(base + L.SV);
        d.dots = (double*)(base + L.dots);
        d.G = (double*)(base + L.G);
        d.H = (double*)(base + L.H);
        d.R = (double*)(base + L.R);
        d.gv = (double*)(base + L.gv);
        d.coef = (float*)(base + L.coef);
        d.y = (double*)(base + L.y);
        d.state = (int*)(base + L.state);
        d.scal = (double*)(base + L.scal);
        d.om1t = (const float*)(base + L.ot1);
        d.om1th = (const bf16_t*)(base + L.ot1h);
        d.om2t = (const float*)(base + L.ot2);
        d.om3t = (const float*)(base + L.ot3);
    }
}

// Host-to-device copies of a plan's descriptors, in stream order.  Under
// stream capture they travel by value as kernel arguments (3 KB per launch),
// so that every replay of the graph writes the captured contents.  Otherwise
// one asynchronous copy from a pinned staging buffer: four buffers per
// device in turn, each reused only once the event recorded behind its last
// copy has completed.
struct Blob {
    unsigned char b[3072];
};

__global__ void k_store(Blob blob, unsigned char* dst, int nbytes) {
    for (int i = threadIdx.x; i < nbytes; i += blockDim.x) dst[i] = blob.b[i];
}

constexpr int STAGE_DEVICES = 16, STAGE_SLOTS = 4;
struct Staging {
    std::mutex mu;
    void* host[STAGE_DEVICES][STAGE_SLOTS] = {};
    size_t cap[STAGE_DEVICES][STAGE_SLOTS] = {};
    hipEvent_t ev[STAGE_DEVICES][STAGE_SLOTS] = {};
    int next[STAGE_DEVICES] = {};
};
Staging g_staging;
// set around the calls of an entry point that may not allocate (the staging
// buffers are allocated on first use): its uploads go by value
thread_local bool t_upload_by_value = false;

int upload_by_value(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const unsigned char* p = (const unsigned char*)src;
    for (size_t off = 0; off < bytes; off += sizeof(Blob)) {
        Blob blob;
        const size_t nb = bytes - off < sizeof(Blob) ? bytes - off : sizeof(Blob);
        std::memcpy(blob.b, p + off, nb);
        hipLaunchKernelGGL(k_store, dim3(1), dim3(256), 0, s, blob, (unsigned char*)dst + off, (int)nb);
    }
    return hipGetLastError() == hipSuccess ? RTG_OK : RTG_E_HIP;
}

int upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return RTG_E_HIP;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RTG_E_HIP;
    if (t_upload_by_value || cs != hipStreamCaptureStatusNone || dev < 0 || dev >= STAGE_DEVICES)
        return upload_by_value(dst, src, bytes, s);
    std::lock_guard<std::mutex> lock(g_staging.mu);
    const int k = g_staging.next[dev];
    g_staging.next[dev] = (k + 1) % STAGE_SLOTS;
    hipEvent_t& ev = g_staging.ev[dev][k];
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return RTG_E_HIP;
    if (hipEventSynchronize(ev) != hipSuccess) return RTG_E_HIP;   // the buffer's previous copy is done
    void*& h = g_staging.host[dev][k];
    if (g_staging.cap[dev][k] < bytes) {
        if (h) (void)hipHostFree(h);
        h = nullptr;
        g_staging.cap[dev][k] = 0;
        const size_t cap = std::max<size_t>(bytes, 64 << 10);
        if (hipHostMalloc(&h, cap, hipHostMallocDefault) != hipSuccess) return RTG_E_HIP;
        g_staging.cap[dev][k] = cap;
    }
    std::memcpy(h, src, bytes);
    if (hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return RTG_E_HIP;
    return hipEventRecord(ev, s) == hipSuccess ? RTG_OK : RTG_E_HIP;
}

struct Plan {
    Desc* d_desc;
    int* d_starts;   // NKIND x (count + 1)
    int total[NKIND];
    int rmax;
    int l1max;
    int compose_max;   // largest entry count of the composed matrices (mode 1 padded to operand tiles)
    int phi_jt;        // output channels per operator tile (one choice per batch)
    bool step_ok;      // the fused step kernel applies (32-bit byte offsets into a basis vector)
    bool lazy_v1;      // V_1 stored unnormalised (Desc::lazy_v1)
    int toeplitz;      // every problem's bands are Toeplitz
    int unsketched;    // every problem's sketch is the identity (a batch is all one or all the other)
    int stencil;       // every problem's operator is a general PSF (all or none)
    int phi_dma;       // operator slab loads: 1 = 16-byte (float32 inputs below 2^31 bytes),
                       // 2 = also asynchronous (and at most three channels), 0 = single-word
    int phi_toep;      // operator: Toeplitz taps in registers
    int step_toep;     // fused step: Toeplitz taps
    int tile_rows;     // sketch tiles per wave of the tile kernel (2 where they fit, or 4)
    int step_rows;     // the same for the fused step
    int skbf;          // sketch contractions on bfloat16 operands (every problem's descriptor says so)
    Desc* d_desc_r;    // restart cycles: the descriptors with X0 = X (null without restarts)
    int persist;       // the Arnoldi process as one persistent launch
    int* d_sched;      // its scheduling words (SCH_WORDS ints)
    int qfirst[NKIND][9];   // its XCD queues: first tile of each queue's problems per kind
};

// descs holds nsides groups of count problems (the same shapes in each group);
// with restart, the restart-cycle copies (X0 = X, R0 from W) follow them.
// tune: the launch shapes (resolved, no -1), clamped to what the batch can
// use; null for the library defaults.
int build_plan(std::vector<Desc>& descs, void* ws, hipStream_t s, Plan& plan, int nsides = 1,
               bool restart = false, const rtg_tune* tune = nullptr, bool solve = false) {
    const int count = (int)descs.size() / nsides;
    std::vector<int> starts((size_t)NKIND * (count + 1), 0);
    int maxJ = 1;
    for (auto& d : descs) maxJ = std::max(maxJ, d.J);
    plan.phi_jt = (tune && (tune->phi_jt == 4 || tune->phi_jt == 8)) ? tune->phi_jt : phi_jt(maxJ);
    for (auto& d : descs)
        if (d.ntile[KIND_PHI] > 0) d.ntile[KIND_PHI] = phi_tiles(d.I1, d.I2, d.J, plan.phi_jt);
    // sketched-Gram chunks: at least the default (the dots area of the
    // workspace holds the default's workgroup count), at most 4096 finished
    // values per workgroup
    for (auto& d : descs) {
        d.gram_ch = 0;
        if (!tune || tune->gram_pairs <= 0 || d.unsketched || gram_split(d.l3, d.J, d.n_i2t)) continue;
        const int def = gram_pairs_per_block(d.l3, d.J, d.n_i2t);
        const int ch = std::max(def, std::min(tune->gram_pairs, 4096 / std::max(d.l3, 1)));
        if (ch == def) continue;
        d.gram_ch = ch;
        d.ntile[KIND_GRAM] = (d.l1 * d.l2 + ch - 1) / ch;
    }
    plan.rmax = 1;
    for (int k = 0; k < NKIND; ++k) {
        int acc = 0;
        for (int p = 0; p < count; ++p) {
            starts[(size_t)k * (count + 1) + p] = acc;
            acc += descs[p].ntile[k];
        }
        starts[(size_t)k * (count + 1) + count] = acc;
        plan.total[k] = acc;
    }
    // the persistent launch's XCD queues: problems in eight contiguous
    // groups of about equal element counts
    {
        long long ntot = 0;
        for (int p = 0; p < count; ++p) ntot += descs[p].n;
        int p = 0;
        long long acc = 0;
        for (int x = 0; x <= 8; ++x) {
            const long long cut = ntot * x / 8;
            while (p < count && (x == 8 || acc + descs[p].n / 2 < cut)) acc += descs[p++].n;
            for (int k = 0; k < NKIND; ++k) plan.qfirst[k][x] = starts[(size_t)k * (count + 1) + p];
        }
    }
    plan.l1max = 1;
    plan.compose_max = 1;
    plan.step_ok = true;
    plan.toeplitz = 1;
    plan.unsketched = descs.empty() ? 0 : descs[0].unsketched;
    plan.stencil = (!descs.empty() && descs[0].st) ? 1 : 0;
    plan.phi_dma = 2;
    for (auto& d : descs) {
        if (d.unsketched != plan.unsketched) return RTG_E_ARG;
        if ((d.st != nullptr) != (plan.stencil != 0)) return RTG_E_ARG;
        if (d.n * 4 > 0x7FFFFFFFll) plan.phi_dma = 0;
        else if (d.J > 3) plan.phi_dma = std::min(plan.phi_dma, 1);
        if (d.unsketched && d.n * 4 > 0x7FFFFFFFll) return RTG_E_SHAPE;
        plan.toeplitz = plan.toeplitz && d.toeplitz;
        plan.step_ok = plan.step_ok && d.n * 2 <= 0x7FFFFFFFll &&
                       frag_elems(d.l1, d.I1, FRAG_K_BF16) * 4 <= 0x7FFFFFFFull && d.a1p[0] != nullptr;
        plan.rmax = std::max(plan.rmax, std::max(d.r1, d.r2));
        if (!d.unsketched) plan.l1max = std::max(plan.l1max, d.l1);
        plan.compose_max = std::max(plan.compose_max, (int)compose_mode1_entries(d.l1, d.I1) + d.l2 * d.I2 + d.l3 * d.J);
    }
    // one pass over R0 forms and sketches V_1 (unnormalised) where the
    // basis stays internal (a solve) and the fused step forms the rest
    plan.lazy_v1 = solve && nsides == 1 && !restart && !plan.unsketched && !plan.stencil && plan.step_ok &&
                   !descs.empty();
    for (auto& d : descs) plan.lazy_v1 = plan.lazy_v1 && d.bf16 && !d.gk;
    for (auto& d : descs) d.lazy_v1 = plan.lazy_v1 ? 1 : 0;
    plan.phi_toep = plan.toeplitz;
    plan.step_toep = plan.toeplitz;
    plan.tile_rows = 2;
    plan.step_rows = 2;
    plan.skbf = descs.empty() ? 0 : descs[0].skbf;
    if (tune) {
        if (tune->phi_slab >= 0) plan.phi_dma = std::min(plan.phi_dma, tune->phi_slab);
        if (tune->phi_toeplitz >= 0) plan.phi_toep = plan.toeplitz && tune->phi_toeplitz;
        if (tune->step_toeplitz >= 0) plan.step_toep = plan.toeplitz && tune->step_toeplitz;
        if (tune->tile_rows == 4) plan.tile_rows = 4;
        if (tune->step_rows == 4) plan.step_rows = 4;
    }
    // the persistent launch: sketched separable RTG-GMRES with a float32
    // basis (either product form), 16-byte operator slabs, one tile for all
    // channels
    plan.persist = tune && tune->persist == 1 && nsides == 1 && !plan.unsketched && !plan.stencil &&
                   plan.phi_jt == 4 && plan.phi_dma >= 1 && !descs.empty() && !descs[0].bf16;
    char* base = (char*)ws;
    plan.d_desc = (Desc*)base;
    plan.d_desc_r = nullptr;
    const size_t nd = descs.size();
    plan.d_starts = (int*)(base + align_up(nd * (restart ? 2 : 1) * sizeof(Desc)));
    plan.d_sched = (int*)((char*)plan.d_starts + align_up((size_t)NKIND * (count + 1) * sizeof(int)));
    // descriptors, the restart cycles' copies and the prefix tables as one
    // image of the region they occupy: a single upload
    const size_t starts_off = (size_t)((char*)plan.d_starts - base);
    std::vector<unsigned char> image(starts_off + starts.size() * sizeof(int), 0);
    std::memcpy(image.data(), descs.data(), nd * sizeof(Desc));
    if (restart) {
        std::vector<Desc> rd(descs);
        for (auto& d : rd) {
            d.X0 = d.X;
            d.R0src = d.W;
        }
        plan.d_desc_r = plan.d_desc + nd;
        std::memcpy(image.data() + nd * sizeof(Desc), rd.data(), nd * sizeof(Desc));
    }
    std::memcpy(image.data() + starts_off, starts.data(), starts.size() * sizeof(int));
    return upload(base, image.data(), image.size(), s);
}

const int* starts_of(const Plan& plan, int kind, int count) {
    return plan.d_starts + (size_t)kind * (count + 1);
}

#define RTG_HIP(call)                                   \
    do {                                                \
        if ((call) != hipSuccess) return RTG_E_HIP;     \
    } while (0)

// ---- optional event timing of launches (measurement facility)
constexpr int NTIMED = 6;   // 0 operator, 1 tile, 2 gram, 3 solve, 4 step, 5 persistent Arnoldi
struct EventTiming {
    int mask = 0;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> rec[NTIMED];
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        // timing-only events: recording one needs no system-scope release
        // (a cache write-back and invalidation before the next launch, which
        // would otherwise sit between every pair of timed launches)
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        return e;
    }
};
EventTiming g_timing;

// polls of a cross-workgroup wait in the persistent launch before it is abandoned
std::atomic<int> g_wait_limit{1 << 22};

struct TimedLaunch {
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(int k, hipStream_t st) : kind(k), s(st) {
        if (g_timing.mask & (1 << kind)) {
            a = g_timing.get();
            b = g_timing.get();
            if (a && b) (void)hipEventRecord(a, s);
        }
    }
    ~TimedLaunch() {
        if (a && b) {
            (void)hipEventRecord(b, s);
            g_timing.rec[kind].push_back({a, b});
        }
    }
};
#define RTG_TIMED_ON(kind, strm, call)                   \
    do {                                                 \
        TimedLaunch _tl((kind), (strm));                 \
        if ((call) != hipSuccess) return RTG_E_HIP;      \
    } while (0)
#define RTG_TIMED(kind, call) RTG_TIMED_ON(kind, s, call)

// Arnoldi loop + (optionally) solve and assembly for a prepared plan.
// cycle > 0: a restart cycle of restarted RTG-GMRES, on the descriptor copies
// whose X0 is the output X (R0 = C - Phi(X)).
int run_solver(const Plan& plan, int count, int mmax, int bf16, bool any_x0, bool solve,
               bool last_newv, hipStream_t s, int cycle = 0) {
    const Desc* dd = cycle > 0 ? plan.d_desc_r : plan.d_desc;
    if (cycle > 0) any_x0 = true;
    const int* sp = starts_of(plan, KIND_PHI, count);
    const int* st = starts_of(plan, KIND_TILE, count);
    const int* sg = starts_of(plan, KIND_GRAM, count);
    RTG_HIP(launch_init(dd, count, s, cycle, plan.persist ? plan.d_sched : nullptr));
    if (plan.unsketched) {
        // Identity sketch (unsketched global GMRES, the Omega = I form of the
        // method): W = Phi(V_j) is formed first, the Gram kernel takes the
        // Frobenius products of the full tensors, and the tile kernel forms
        // V_{j+1} without sketching.
        const int us = 1;
        if (any_x0)
            RTG_TIMED(0, launch_phi(dd, sp, count, plan.total[KIND_PHI], PS_X0, 0, plan.rmax, plan.phi_jt, 0,
                                    s, plan.stencil, plan.phi_dma, plan.phi_toep));
        RTG_TIMED(2, launch_gram(dd, sg, count, plan.total[KIND_GRAM], GM_START, cycle, nullptr, s, us));
        RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_NEWV, 0, 0, bf16, 0, plan.l1max, s, 0, plan.tile_rows, plan.skbf));
        for (int j = 1; j <= mmax; ++j) {
            RTG_TIMED(0, launch_phi(dd, sp, count, plan.total[KIND_PHI], PS_BASIS, j - 1, plan.rmax,
                                    plan.phi_jt, bf16, s, plan.stencil, plan.phi_dma, plan.phi_toep));
            RTG_TIMED(2, launch_gram(dd, sg, count, plan.total[KIND_GRAM], GM_STEP, j, nullptr, s, us));
            if (j < mmax || last_newv)
                RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_NEWV, j, j, bf16, 0,
                                         plan.l1max, s, 0, plan.tile_rows, plan.skbf));
        }
        if (solve) {
            RTG_TIMED(3, launch_solve(dd, count, mmax, s));
            RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_ASSEMBLE, 0, 0, bf16, 0,
                                     plan.l1max, s, 0, plan.tile_rows, plan.skbf));
        }
        return RTG_OK;
    }
    if (plan.stencil) {
        // General PSF: no composed sketch matrices.  Step j forms W = Phi(V_j),
        // sketches W, then the Gram step and V_{j+1} with its sketch.
        if (any_x0)
            RTG_TIMED(0, launch_phi(dd, sp, count, plan.total[KIND_PHI], PS_X0, 0, plan.rmax, plan.phi_jt, 0,
                                    s, 1, plan.phi_dma, plan.phi_toep));
        RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_SKETCH_SRC, 0, 0, bf16, 0,
                                 plan.l1max, s, 0, plan.tile_rows, plan.skbf));
        RTG_TIMED(2, launch_gram(dd, sg, count, plan.total[KIND_GRAM], GM_START, cycle, nullptr, s));
        RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_NEWV, 0, 0, bf16, 0, plan.l1max, s, 0, plan.tile_rows, plan.skbf));
        for (int j = 1; j <= mmax; ++j) {
            RTG_TIMED(0, launch_phi(dd, sp, count, plan.total[KIND_PHI], PS_BASIS, j - 1, plan.rmax,
                                    plan.phi_jt, bf16, s, 1, plan.phi_dma, plan.phi_toep));
            RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_SKETCH_W, 0, 0, bf16, 0,
                                     plan.l1max, s, 0, plan.tile_rows, plan.skbf));
            RTG_TIMED(2, launch_gram(dd, sg, count, plan.total[KIND_GRAM], GM_STEP, j, nullptr, s));
            if (j < mmax || last_newv)
                RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_NEWV, j, j, bf16, 0,
                                         plan.l1max, s, 0, plan.tile_rows, plan.skbf));
        }
        if (solve) {
            RTG_TIMED(3, launch_solve(dd, count, mmax, s));
            RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_ASSEMBLE, 0, 0, bf16, 0,
                                     plan.l1max, s, 0, plan.tile_rows, plan.skbf));
        }
        return RTG_OK;
    }
    if (cycle == 0) RTG_HIP(launch_compose(dd, count, plan.compose_max, s));   // restart cycles reuse them
    if (plan.persist) {
        // the start and every step of every problem: one launch
        PersistArgs a{};
        a.descs = dd;
        a.starts[KIND_PHI] = sp;
        a.starts[KIND_TILE] = st;
        a.starts[KIND_GRAM] = sg;
        a.count = count;
        std::memcpy(a.qfirst, plan.qfirst, sizeof(a.qfirst));
        a.any_x0 = any_x0 ? 1 : 0;
        a.cycle = cycle;
        a.sched = plan.d_sched;
        a.wait_limit = g_wait_limit.load();
        a.steps = mmax;
        a.full = last_newv ? mmax : mmax - 1;   // steps that form V_{j+1}
        const long long tp = plan.total[KIND_PHI], tt = plan.total[KIND_TILE], tg = plan.total[KIND_GRAM];
        const long long total = (any_x0 ? tp : 0) + 2 * tt + tg + (long long)mmax * tg + (long long)a.full * (tp + tt);
        if (total > 0x3FFFFFFFLL) return RTG_E_SHAPE;
        RTG_TIMED(5, launch_persist(a, plan.rmax, plan.phi_toep, plan.skbf, s));
        if (solve) {
            RTG_TIMED(3, launch_solve(dd, count, mmax, s));
            RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_ASSEMBLE, 0, 0, bf16, 0, plan.l1max, s, 0,
                                     plan.tile_rows, plan.skbf));
        }
        return RTG_OK;
    }
    const bool lazy = plan.lazy_v1 && cycle == 0;
    // (a bfloat16 basis stored unnormalised: the operator kernel stores R0 =
    // C - Phi(X0) rounded to bfloat16 as V_1 itself)
    if (any_x0) RTG_TIMED(0, launch_phi(dd, sp, count, plan.total[KIND_PHI], lazy ? PS_X0_V1 : PS_X0, 0, plan.rmax, plan.phi_jt, 0, s, 0, plan.phi_dma, plan.phi_toep));
    if (lazy) {
        // V_1 = R0 (scale 1, set by the init kernel) with both its sketches
        // in one pass (stored there too where X0 is absent, R0 = C); the
        // start step takes beta from S(V_1)
        RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_NEWV1, 0, 0, bf16, 0, plan.l1max, s, 0, plan.tile_rows, plan.skbf));
        RTG_TIMED(2, launch_gram(dd, sg, count, plan.total[KIND_GRAM], GM_START, cycle, nullptr, s));
    } else {
        RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_SKETCH_SRC, 0, 0, bf16, 0, plan.l1max, s, 0, plan.tile_rows, plan.skbf));
        RTG_TIMED(2, launch_gram(dd, sg, count, plan.total[KIND_GRAM], GM_START, cycle, nullptr, s));
        RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_NEWV, 0, 0, bf16, 0, plan.l1max, s, 0, plan.tile_rows, plan.skbf));
    }
    for (int j = 1; j <= mmax; ++j) {
        // S(V_j) and S(Phi(V_j)) come from the pass that formed V_j.  With a
        // bfloat16 basis the step kernel recomputes Phi(V_j) tile by tile (W
        // is never stored); with a float32 basis W is formed by the operator
        // kernel and read by the multi-AXPY tile kernel, which measured faster
        // there (the fused kernel's float32 variant runs at lower occupancy).
        // The same two kernels serve a bfloat16 basis whose vectors reach
        // 2^31 bytes (the fused kernel addresses them with 32-bit offsets).
        RTG_TIMED(2, launch_gram(dd, sg, count, plan.total[KIND_GRAM], GM_STEP, j, nullptr, s));
        if (j < mmax || last_newv) {
            if (bf16 && plan.step_ok) {
                RTG_TIMED(4, launch_step(dd, st, count, plan.total[KIND_TILE], j, plan.rmax, bf16, plan.l1max,
                                         plan.step_toep, s, plan.step_rows));
            } else {
                RTG_TIMED(0, launch_phi(dd, sp, count, plan.total[KIND_PHI], PS_BASIS, j - 1, plan.rmax,
                                        plan.phi_jt, bf16, s, 0, plan.phi_dma, plan.phi_toep));
                RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_NEWV, j, j, bf16, 0,
                                         plan.l1max, s, 0, plan.tile_rows, plan.skbf));
            }
        }
    }
    if (solve) {
        RTG_TIMED(3, launch_solve(dd, count, mmax, s));
        RTG_TIMED(1, launch_tile(dd, st, count, plan.total[KIND_TILE], TM_ASSEMBLE, 0, 0, bf16, 0, plan.l1max, s, 0, plan.tile_rows, plan.skbf));
    }
    return RTG_OK;
}

// Sketched Block Golub-Kahan (Sec. 4.5) for a prepared two-sided plan:
// descriptors [0, count) are the V sides (operator Phi), [count, 2 count)
// the U sides (operator Phi^T).  Each half-step is the sketched norm of the
// next tensor in sketch space (Gram kernel, from the composed sketch of the
// newest tensor and the other side's stored sketch), the operator applied to
// the newest tensor (into W), and the one-term AXPY that stores the next
// tensor with its two sketches.  The last column needs no U_{m+1}.
int run_gk(const Plan& plan, int count, int mmax, int bf16, bool any_x0, bool solve, hipStream_t s) {
    const int* sp = starts_of(plan, KIND_PHI, count);
    const int* st = starts_of(plan, KIND_TILE, count);
    const int* sg = starts_of(plan, KIND_GRAM, count);
    const Desc* dV = plan.d_desc;
    const Desc* dU = plan.d_desc + count;
    const int tp = plan.total[KIND_PHI], tt = plan.total[KIND_TILE], tg = plan.total[KIND_GRAM];
    RTG_HIP(launch_init(dV, count, s));
    RTG_HIP(launch_compose(plan.d_desc, 2 * count, plan.compose_max, s));
    if (any_x0) RTG_TIMED(0, launch_phi(dV, sp, count, tp, PS_X0, 0, plan.rmax, plan.phi_jt, 0, s, 0, plan.phi_dma, plan.phi_toep));
    // beta_1 = ||R0||_Theta, U_1 = R0 / beta_1 (with S(U_1) and S(Phi^T(U_1)))
    RTG_TIMED(1, launch_tile(dU, st, count, tt, TM_SKETCH_SRC, 0, 0, bf16, 0, plan.l1max, s, 0, plan.tile_rows));
    RTG_TIMED(2, launch_gram(dU, sg, count, tg, GM_START, 0, nullptr, s));
    RTG_TIMED(1, launch_tile(dU, st, count, tt, TM_NEWV, 0, 0, bf16, 0, plan.l1max, s, 0, plan.tile_rows));
    for (int c = 1; c <= mmax; ++c) {
        // alpha_c; V_c = (Phi^T(U_c) - beta_c V_{c-1}) / alpha_c
        RTG_TIMED(2, launch_gram(dU, sg, count, tg, GM_GK, c, nullptr, s));
        RTG_TIMED(0, launch_phi(dU, sp, count, tp, PS_BASIS, c - 1, plan.rmax, plan.phi_jt, bf16, s, 0, plan.phi_dma, plan.phi_toep));
        RTG_TIMED(1, launch_tile(dV, st, count, tt, TM_GKNEW, c - 1, c - 1, bf16, 0, plan.l1max, s,
                                 c >= 2 ? c - 2 : 0));
        // beta_{c+1}, column c of B, Givens and stop test; U_{c+1} = (Phi(V_c) - alpha_c U_c) / beta_{c+1}
        RTG_TIMED(2, launch_gram(dV, sg, count, tg, GM_GK, c, nullptr, s));
        if (c < mmax || !solve) {   // the bidiagonalisation alone also forms U_{m+1}
            RTG_TIMED(0, launch_phi(dV, sp, count, tp, PS_BASIS, c - 1, plan.rmax, plan.phi_jt, bf16, s, 0, plan.phi_dma, plan.phi_toep));
            RTG_TIMED(1, launch_tile(dU, st, count, tt, TM_GKNEW, c, c, bf16, 0, plan.l1max, s, c - 1, plan.tile_rows));
        }
    }
    if (solve) {
        RTG_TIMED(3, launch_solve(dV, count, mmax, s));
        RTG_TIMED(1, launch_tile(dV, st, count, tt, TM_ASSEMBLE, 0, 0, bf16, 0, plan.l1max, s, 0, plan.tile_rows));
    }
    return RTG_OK;
}

int validate_params(const rtg_params* prm) {
    if (!prm) return RTG_E_ARG;
    if (prm->basis_dtype != RTG_F32 && prm->basis_dtype != RTG_BF16 && prm->basis_dtype != RTG_F32_BF16)
        return RTG_E_ARG;
    // the mixed form (float32 basis, bfloat16 sketch products) is RTG-GMRES only
    if (prm->basis_dtype == RTG_F32_BF16 && prm->method != RTG_METHOD_GMRES) return RTG_E_ARG;
    if (prm->mu_rule != RTG_MU_DISCREPANCY && prm->mu_rule != RTG_MU_GCV) return RTG_E_ARG;
    if (prm->method != RTG_METHOD_GMRES && prm->method != RTG_METHOD_GOLUB_KAHAN) return RTG_E_ARG;
    // restarts: a tolerance eps (stop_res) is what ends them; RTG-GMRES only
    if (prm->restarts < 0 || prm->restarts > 10000) return RTG_E_ARG;
    if (prm->restarts > 0 && (!(prm->stop_res > 0.0) || prm->method != RTG_METHOD_GMRES)) return RTG_E_ARG;
    if (prm->mu < 0.0 && prm->mu_rule == RTG_MU_DISCREPANCY && !(prm->delta >= 0.0 && prm->eta > 0.0))
        return RTG_E_ARG;
    if (!(prm->bd_tol >= 0.0)) return RTG_E_ARG;
    return RTG_OK;
}

void set_params(Desc& d, const rtg_params* prm) {
    d.mu_fixed = prm->mu >= 0.0 ? 1 : 0;
    d.mu_rule = prm->mu_rule;
    d.mu = prm->mu >= 0.0 ? prm->mu : 0.0;
    d.delta = prm->delta;
    d.eta = prm->eta;
    d.stop_res = prm->stop_res;
    d.bd_tol = prm->bd_tol;
    d.restarts = prm->restarts;
}

}  // namespace

extern "C" {

const char* rtg_status_string(int status) {
    switch (status) {
        case RTG_OK: return "ok";
        case RTG_E_ARG: return "invalid argument";
        case RTG_E_SHAPE: return "inconsistent or unsupported sizes";
        case RTG_E_HIP: return "HIP runtime error";
        case RTG_E_NOMEM: return "device allocation failed";
        case RTG_E_WORKSPACE: return "workspace too small";
        default: return "unknown status";
    }
}

static int setup_op(int I1, int I2, int J, const float* a1_band, int r1, const float* a2_band,
                    int r2, const float* b_band, int rB, rtg_op* out) {
    if (!out || !a1_band || !a2_band || !b_band) return RTG_E_ARG;
    *out = nullptr;
    if (I1 < 8 || I2 < 1 || J < 1 || (I1 % 8) != 0) return RTG_E_SHAPE;
    if (r1 < 0 || r2 < 0 || rB < 0 || r1 > RMAX_SPATIAL || r2 > RMAX_SPATIAL || rB > RMAX_B) return RTG_E_SHAPE;
    if (r1 >= I1 || (r2 >= I2 && I2 > 1) || (rB >= J && J > 1)) return RTG_E_SHAPE;
    rtg_op_s* op = new rtg_op_s{I1, I2, J, r1, r2, rB, nullptr, nullptr, nullptr, nullptr, nullptr,
                                {nullptr, nullptr, nullptr}, 0, nullptr, nullptr};
    // Toeplitz bands (a convolution with zero boundary conditions, such as the
    // blurs of Sec. 5): A[i, i + dd] the same for every row i with i + dd in
    // range, compared bit for bit.  Entries pointing outside the matrix are
    // never used (they meet the zero boundary) and are not compared.
    std::vector<float> taps(2 * (2 * RMAX_SPATIAL + 1), 0.f);
    auto toeplitz_taps = [](const float* band, int I, int r, float* t) {
        const int w = 2 * r + 1;
        for (int dd = -r; dd <= r; ++dd) {
            const int i0 = dd >= 0 ? 0 : -dd;            // first row where column i0 + dd exists
            if (i0 + dd >= I) { t[r + dd] = 0.f; continue; }
            const float v = band[(size_t)i0 * w + r + dd];
            for (int i = i0; i < I && i + dd < I; ++i)
                if (std::memcmp(band + (size_t)i * w + r + dd, &v, sizeof(float)) != 0) return false;
            t[r + dd] = v;
        }
        return true;
    };
    op->toeplitz = (toeplitz_taps(a1_band, I1, r1, taps.data()) &&
                    toeplitz_taps(a2_band, I2, r2, taps.data() + 2 * RMAX_SPATIAL + 1)) ? 1 : 0;
    const size_t n1 = (size_t)I1 * (2 * r1 + 1), n2 = (size_t)I2 * (2 * r2 + 1), nb = (size_t)J * (2 * rB + 1);
    if (hipMalloc(&op->a1, n1 * 4) != hipSuccess || hipMalloc(&op->a2, n2 * 4) != hipSuccess ||
        hipMalloc(&op->bb, nb * 4) != hipSuccess || hipMalloc(&op->a1t, n1 * 4) != hipSuccess ||
        hipMalloc(&op->a2t, n2 * 4) != hipSuccess) {
        rtg_destroy_operator(op);
        return RTG_E_NOMEM;
    }
    auto transpose_band = [](const float* band, int I, int r) {
        const int w = 2 * r + 1;
        std::vector<float> t((size_t)I * w);
        for (int i = 0; i < I; ++i)
            for (int k = 0; k < w; ++k) t[(size_t)k * I + i] = band[(size_t)i * w + k];
        return t;
    };
    const std::vector<float> a1t = transpose_band(a1_band, I1, r1), a2t = transpose_band(a2_band, I2, r2);
    for (int k = 0; k < 3; ++k) {
        const int R = 4 * (k + 1), WP = ((2 * R + 1) + 3) / 4 * 4;
        std::vector<float> pad((size_t)I1 * WP, 0.f);
        if (r1 <= R)
            for (int i = 0; i < I1; ++i)
                for (int dd = -r1; dd <= r1; ++dd) pad[(size_t)i * WP + R + dd] = a1_band[(size_t)i * (2 * r1 + 1) + r1 + dd];
        if (hipMalloc(&op->a1p[k], pad.size() * 4) != hipSuccess) {
            rtg_destroy_operator(op);
            return RTG_E_NOMEM;
        }
        if (hipMemcpy(op->a1p[k], pad.data(), pad.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
            rtg_destroy_operator(op);
            return RTG_E_HIP;
        }
    }
    if (hipMalloc(&op->taps, taps.size() * 4) != hipSuccess) {
        rtg_destroy_operator(op);
        return RTG_E_NOMEM;
    }
    if (hipMemcpy(op->taps, taps.data(), taps.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        rtg_destroy_operator(op);
        return RTG_E_HIP;
    }
    if (hipMemcpy(op->a1, a1_band, n1 * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->a2, a2_band, n2 * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->bb, b_band, nb * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->a1t, a1t.data(), n1 * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->a2t, a2t.data(), n2 * 4, hipMemcpyHostToDevice) != hipSuccess) {
        rtg_destroy_operator(op);
        return RTG_E_HIP;
    }
    *out = op;
    return RTG_OK;
}

int rtg_setup_operator(int I1, int I2, int J, const float* a1_band, int r1, const float* a2_band,
                       int r2, const float* b_band, int rB, rtg_op* out) {
    int rc = setup_op(I1, I2, J, a1_band, r1, a2_band, r2, b_band, rB, out);
    if (rc) return rc;
    // the adjoint operator Phi^T (Golub-Kahan): every band transposed,
    // M^T[i, i + dd] = M[i + dd, i], zero where row i + dd leaves the matrix
    auto transposed = [](const float* band, int I, int r) {
        const int w = 2 * r + 1;
        std::vector<float> t((size_t)I * w, 0.f);
        for (int i = 0; i < I; ++i)
            for (int dd = -r; dd <= r; ++dd)
                if (i + dd >= 0 && i + dd < I) t[(size_t)i * w + r + dd] = band[(size_t)(i + dd) * w + r - dd];
        return t;
    };
    const std::vector<float> a1 = transposed(a1_band, I1, r1), a2 = transposed(a2_band, I2, r2),
                             b = transposed(b_band, J, rB);
    rtg_op adj = nullptr;
    rc = setup_op(I1, I2, J, a1.data(), r1, a2.data(), r2, b.data(), rB, &adj);
    if (rc) {
        rtg_destroy_operator(*out);
        *out = nullptr;
        return rc;
    }
    (*out)->adj = adj;
    return RTG_OK;
}

int rtg_setup_operator_psf(int I1, int I2, int J, const float* psf, int r, const float* b_band, int rB,
                           rtg_op* out) {
    if (!out || !psf || !b_band) return RTG_E_ARG;
    *out = nullptr;
    if (I1 < 8 || I2 < 1 || J < 1 || (I1 % 8) != 0) return RTG_E_SHAPE;
    if (r < 0 || rB < 0 || r > RMAX_SPATIAL || rB > RMAX_B) return RTG_E_SHAPE;
    if (r >= I1 || (r >= I2 && I2 > 1) || (rB >= J && J > 1)) return RTG_E_SHAPE;
    rtg_op_s* op = new rtg_op_s{I1, I2, J, r, r, rB, nullptr, nullptr, nullptr, nullptr, nullptr,
                                {nullptr, nullptr, nullptr}, 0, nullptr, nullptr, nullptr};
    // the weight of X[i1 + a, i2 + b] is P[r - a][r - b] (eq. (57))
    const int w = 2 * r + 1;
    std::vector<float> st((size_t)w * w);
    for (int a = -r; a <= r; ++a)
        for (int b = -r; b <= r; ++b) st[(size_t)(a + r) * w + b + r] = psf[(size_t)(r - a) * w + r - b];
    const size_t nb = (size_t)J * (2 * rB + 1);
    if (hipMalloc(&op->st, st.size() * 4) != hipSuccess || hipMalloc(&op->bb, nb * 4) != hipSuccess) {
        rtg_destroy_operator(op);
        return RTG_E_NOMEM;
    }
    if (hipMemcpy(op->st, st.data(), st.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->bb, b_band, nb * 4, hipMemcpyHostToDevice) != hipSuccess) {
        rtg_destroy_operator(op);
        return RTG_E_HIP;
    }
    *out = op;
    return RTG_OK;
}

int rtg_destroy_operator(rtg_op op) {
    if (!op) return RTG_OK;
    if (op->adj) rtg_destroy_operator(op->adj);
    if (op->st) (void)hipFree(op->st);
    if (op->a1) (void)hipFree(op->a1);
    if (op->a2) (void)hipFree(op->a2);
    if (op->bb) (void)hipFree(op->bb);
    if (op->a1t) (void)hipFree(op->a1t);
    if (op->a2t) (void)hipFree(op->a2t);
    for (int k = 0; k < 3; ++k)
        if (op->a1p[k]) (void)hipFree(op->a1p[k]);
    if (op->taps) (void)hipFree(op->taps);
    delete op;
    return RTG_OK;
}

int rtg_apply_operator(rtg_op op, int x_dtype, const void* X, const float* C, float* Y, void* stream) {
    if (!op || !X || !Y) return RTG_E_ARG;
    if (x_dtype != RTG_F32 && x_dtype != RTG_BF16) return RTG_E_ARG;
    if (launch_phi_single(op->I1, op->I2, op->J, op->r1, op->r2, op->rB, op->a1, op->a2, op->bb, op->st,
                          op->toeplitz ? op->taps : nullptr, X,
                          x_dtype == RTG_BF16, C, Y, (hipStream_t)stream) != hipSuccess)
        return RTG_E_HIP;
    return RTG_OK;
}

static bf16_t host_f2bf(float f) {
    uint32_t x;
    std::memcpy(&x, &f, 4);
    if ((x & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((x >> 16) | 0x40u);
    x += 0x7fffu + ((x >> 16) & 1u);
    return (bf16_t)(x >> 16);
}

int rtg_setup_sketch(int I1, int I2, int J, int l1, int l2, int l3, const float* om1,
                     const float* om2, const float* om3, rtg_sk* out) {
    if (!out) return RTG_E_ARG;
    *out = nullptr;
    if (I1 < 8 || I2 < 1 || J < 1 || (I1 % 8) != 0) return RTG_E_SHAPE;
    if (!om1 && !om2 && !om3) {
        // identity on every mode: the unsketched method, any size (no matrices kept)
        if (l1 != I1 || l2 != I2 || l3 != J) return RTG_E_SHAPE;
        if (I1 >= (1 << 20) || I2 >= (1 << 20)) return RTG_E_SHAPE;
        *out = new rtg_sk_s{I1, I2, J, l1, l2, l3, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 1};
        return RTG_OK;
    }
    if (l1 < 1 || l1 > I1 || l1 > LMAX_SPATIAL || l2 < 1 || l2 > I2 || l2 > LMAX_SPATIAL) return RTG_E_SHAPE;
    if ((!om1 && l1 != I1) || (!om2 && l2 != I2) || (!om3 && l3 != J)) return RTG_E_SHAPE;
    if (om3 && (l3 < 1 || l3 > J || l3 > LMAX_3)) return RTG_E_SHAPE;
    if (!om3 && J > 4096) return RTG_E_SHAPE;
    if (I1 >= (1 << 20) || I2 >= (1 << 20)) return RTG_E_SHAPE;   // 32-bit byte offsets into the sketch matrices
    rtg_sk_s* sk = new rtg_sk_s{I1, I2, J, l1, l2, l3, om3 ? 1 : 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0};
    // identity factors are stored explicitly for modes 1 and 2
    std::vector<float> h1((size_t)l1 * I1, 0.f), h2((size_t)l2 * I2, 0.f);
    if (om1) std::memcpy(h1.data(), om1, h1.size() * 4);
    else for (int i = 0; i < I1; ++i) h1[(size_t)i * I1 + i] = 1.f;
    if (om2) std::memcpy(h2.data(), om2, h2.size() * 4);
    else for (int i = 0; i < I2; ++i) h2[(size_t)i * I2 + i] = 1.f;
    std::vector<bf16_t> h1h(h1.size());
    for (size_t i = 0; i < h1.size(); ++i) h1h[i] = host_f2bf(h1[i]);
    // operand-order copies for the MFMA contractions (zero padding)
    std::vector<float> h1f(frag_elems(l1, I1, FRAG_K_F32), 0.f);
    std::vector<bf16_t> h1hf(frag_elems(l1, I1, FRAG_K_BF16), 0);
    const int nkf = frag_nkb(I1, FRAG_K_F32), nkh = frag_nkb(I1, FRAG_K_BF16);
    for (int a = 0; a < l1; ++a)
        for (int i = 0; i < I1; ++i) {
            h1f[frag_index(a, i, nkf, FRAG_K_F32)] = h1[(size_t)a * I1 + i];
            h1hf[frag_index(a, i, nkh, FRAG_K_BF16)] = h1h[(size_t)a * I1 + i];
        }
    bool ok = hipMalloc(&sk->om1, h1.size() * 4) == hipSuccess &&
              hipMalloc(&sk->om2, h2.size() * 4) == hipSuccess &&
              hipMalloc(&sk->om1h, h1h.size() * 2) == hipSuccess &&
              hipMalloc(&sk->om1f, h1f.size() * 4) == hipSuccess &&
              hipMalloc(&sk->om1hf, h1hf.size() * 2) == hipSuccess &&
              (!om3 || hipMalloc(&sk->om3, (size_t)l3 * J * 4) == hipSuccess);
    if (!ok) {
        rtg_destroy_sketch(sk);
        return RTG_E_NOMEM;
    }
    ok = hipMemcpy(sk->om1, h1.data(), h1.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(sk->om2, h2.data(), h2.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(sk->om1h, h1h.data(), h1h.size() * 2, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(sk->om1f, h1f.data(), h1f.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(sk->om1hf, h1hf.data(), h1hf.size() * 2, hipMemcpyHostToDevice) == hipSuccess &&
         (!om3 || hipMemcpy(sk->om3, om3, (size_t)l3 * J * 4, hipMemcpyHostToDevice) == hipSuccess);
    if (!ok) {
        rtg_destroy_sketch(sk);
        return RTG_E_HIP;
    }
    *out = sk;
    return RTG_OK;
}

int rtg_destroy_sketch(rtg_sk sk) {
    if (!sk) return RTG_OK;
    if (sk->om1) (void)hipFree(sk->om1);
    if (sk->om2) (void)hipFree(sk->om2);
    if (sk->om3) (void)hipFree(sk->om3);
    if (sk->om1h) (void)hipFree(sk->om1h);
    if (sk->om1f) (void)hipFree(sk->om1f);
    if (sk->om1hf) (void)hipFree(sk->om1hf);
    delete sk;
    return RTG_OK;
}

size_t rtg_sketch_workspace_bytes(rtg_sk sk) {
    if (!sk) return 0;
    const int n_i2t = (sk->I2 + TILE_TC - 1) / TILE_TC;
    if (sk->identity) return plan_bytes(1);
    return plan_bytes(1) + align_up((size_t)sk->J * n_i2t * sk->l1 * sk->l2 * sizeof(float));
}

int rtg_sketch(rtg_sk sk, int x_dtype, const void* X, float* SX, void* ws, size_t ws_bytes, void* stream) {
    if (!sk || !X || !SX || !ws) return RTG_E_ARG;
    if (x_dtype != RTG_F32 && x_dtype != RTG_BF16) return RTG_E_ARG;
    if (!aligned16(X) || !aligned16(ws)) return RTG_E_ARG;
    if (ws_bytes < rtg_sketch_workspace_bytes(sk)) return RTG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (sk->identity) {      // S(X) = X, same column-major order
        if (x_dtype != RTG_F32) return RTG_E_ARG;
        RTG_HIP(hipMemcpyAsync(SX, X, (size_t)sk->I1 * sk->I2 * sk->J * sizeof(float), hipMemcpyDeviceToDevice, s));
        return RTG_OK;
    }
    rtg_op_s dummy{sk->I1, sk->I2, sk->J, 0, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                   {nullptr, nullptr, nullptr}, 0, nullptr, nullptr};
    Layout L = problem_layout(&dummy, sk, 1, x_dtype == RTG_BF16);
    std::vector<Desc> descs(1);
    fill_desc(descs[0], &dummy, sk, 1, x_dtype == RTG_BF16, nullptr, L);
    descs[0].PW = (float*)((char*)ws + plan_bytes(1));
    descs[0].R0src = X;
    descs[0].src_bf16 = x_dtype == RTG_BF16;
    descs[0].ntile[KIND_PHI] = 0;
    Plan plan;
    int rc = build_plan(descs, ws, s, plan);
    if (rc) return rc;
    RTG_HIP(launch_tile(plan.d_desc, starts_of(plan, KIND_TILE, 1), 1, plan.total[KIND_TILE], TM_SKETCH_SRC,
                        0, 0, x_dtype == RTG_BF16, x_dtype == RTG_BF16, plan.l1max, s, 0, plan.tile_rows));
    RTG_HIP(launch_gram(plan.d_desc, starts_of(plan, KIND_GRAM, 1), 1, plan.total[KIND_GRAM], GM_SKETCH_OUT,
                        0, SX, s));
    return RTG_OK;
}

}  // extern "C"

// ---- the sketch without a caller workspace (rtg_sketch_noalloc)
// Its descriptor, prefix table and per-tile partial sketches live in a
// file-scope device array: every GPU the library runs on holds its own copy
// from the load of the code object to the end of the process.  Host code
// never passes the array's name to a kernel (on the host it only stands in
// for the symbol); it passes the device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.
namespace {
constexpr size_t SKETCH_SCRATCH_BYTES = (size_t)RTG_SKETCH_NOALLOC_MAX_BYTES;
__device__ __align__(256) unsigned char scratch[SKETCH_SCRATCH_BYTES];

struct ScratchTable {
    std::mutex mu;
    std::vector<void*> ptr;   // device address of scratch, per device ordinal
};

ScratchTable& scratch_table() {
    static ScratchTable t;
    return t;
}

int scratch_of_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return RTG_E_HIP;
    ScratchTable& t = scratch_table();
    std::lock_guard<std::mutex> lock(t.mu);
    if ((size_t)dev >= t.ptr.size()) t.ptr.resize((size_t)dev + 1, nullptr);
    if (!t.ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RTG_E_HIP;
        t.ptr[dev] = p;
    }
    *out = t.ptr[dev];
    return RTG_OK;
}
}  // namespace

extern "C" {

int rtg_sketch_noalloc(rtg_sk sk, int x_dtype, const void* X, float* SX, void* stream) {
    if (!sk || !X || !SX) return RTG_E_ARG;
    if (x_dtype != RTG_F32 && x_dtype != RTG_BF16) return RTG_E_ARG;
    if (rtg_sketch_workspace_bytes(sk) > SKETCH_SCRATCH_BYTES) return RTG_E_WORKSPACE;
    void* ws = nullptr;
    const int rc = scratch_of_current_device(&ws);
    if (rc) return rc;
    // the same launches as rtg_sketch, on the device array: nothing in it
    // has to start at zero (the descriptor and the prefix table are uploaded
    // by every call, as kernel arguments, and every tile writes its whole
    // partial sketch)
    struct ByValue {
        ByValue() { t_upload_by_value = true; }
        ~ByValue() { t_upload_by_value = false; }
    } by_value;
    return rtg_sketch(sk, x_dtype, X, SX, ws, SKETCH_SCRATCH_BYTES, stream);
}

size_t rtg_workspace_bytes(rtg_op op, rtg_sk sk, int m, int basis_dtype) {
    if (check_pair(op, sk) || check_m(sk, m)) return 0;
    // (room for the restart-cycle descriptor copy of rtg_solve with restarts)
    return plan_bytes(1, 1, true) + problem_layout(op, sk, m, basis_dtype == RTG_BF16).total;
}

int rtg_workspace_layout(rtg_op op, rtg_sk sk, int m, int basis_dtype, size_t* v_offset, size_t* sv_offset) {
    int rc = check_pair(op, sk);
    if (rc) return rc;
    if ((rc = check_m(sk, m))) return rc;
    Layout L = problem_layout(op, sk, m, basis_dtype == RTG_BF16);
    if (v_offset) *v_offset = plan_bytes(1) + L.V;
    if (sv_offset) *sv_offset = plan_bytes(1) + L.SV;
    return RTG_OK;
}

int rtg_arnoldi(rtg_op op, rtg_sk sk, const float* R0, int m, int basis_dtype, double bd_tol, void* ws,
                size_t ws_bytes, double* H, double* beta, int* m_done, void* stream) {
    int rc = check_pair(op, sk);
    if (rc) return rc;
    if ((rc = check_m(sk, m))) return rc;
    if (!R0 || !ws || !H || !beta || !m_done) return RTG_E_ARG;
    if (basis_dtype != RTG_F32 && basis_dtype != RTG_BF16 && basis_dtype != RTG_F32_BF16) return RTG_E_ARG;
    if (!aligned16(R0) || !aligned16(ws) || !(bd_tol >= 0.0)) return RTG_E_ARG;
    const int bf16 = basis_dtype == RTG_BF16;
    if (ws_bytes < rtg_workspace_bytes(op, sk, m, basis_dtype)) return RTG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Layout L = problem_layout(op, sk, m, bf16);
    std::vector<Desc> descs(1);
    fill_desc(descs[0], op, sk, m, bf16, (char*)ws + plan_bytes(1), L);
    descs[0].R0src = R0;
    descs[0].bd_tol = bd_tol;
    descs[0].m = m;
    descs[0].keep_last = 1;
    descs[0].skbf = basis_dtype != RTG_F32;
    Plan plan;
    if ((rc = build_plan(descs, ws, s, plan))) return rc;
    // the last step also forms V_{m+1} (used by the Arnoldi relation):
    // run one more normalisation than a solve needs
    if ((rc = run_solver(plan, 1, m, bf16, false, false, true, s))) return rc;
    RTG_HIP(launch_finish_arnoldi(plan.d_desc, H, beta, m_done, m, s));
    return RTG_OK;
}

size_t rtg_batch_workspace_bytes(int count, const rtg_problem* probs) {
    if (count < 1 || !probs) return 0;
    const int method = probs[0].params.method;
    bool restart = false;
    for (int p = 0; p < count; ++p) restart = restart || probs[p].params.restarts > 0;
    size_t total = plan_bytes(count, method == RTG_METHOD_GOLUB_KAHAN ? 2 : 1, restart);
    for (int p = 0; p < count; ++p) {
        const rtg_problem& q = probs[p];
        if (check_pair(q.op, q.sk) || check_m(q.sk, q.params.m)) return 0;
        if (q.params.method != method) return 0;
        total += problem_bytes(q.op, q.sk, q.params.m, q.params.basis_dtype == RTG_BF16, method);
    }
    return total;
}

size_t rtg_gk_workspace_bytes(rtg_op op, rtg_sk sk, int m, int basis_dtype) {
    if (check_pair(op, sk) || check_m(sk, m)) return 0;
    return plan_bytes(1, 2) + problem_bytes(op, sk, m, basis_dtype == RTG_BF16, RTG_METHOD_GOLUB_KAHAN);
}

int rtg_gk_workspace_layout(rtg_op op, rtg_sk sk, int m, int basis_dtype, size_t* v_offset, size_t* u_offset) {
    int rc = check_pair(op, sk);
    if (rc) return rc;
    if ((rc = check_m(sk, m))) return rc;
    const int bf16 = basis_dtype == RTG_BF16;
    const Layout L = problem_layout(op, sk, m, bf16);
    const GKExtra E = gk_extra_layout(op, sk, m, bf16);
    if (v_offset) *v_offset = plan_bytes(1, 2) + L.V;
    if (u_offset) *u_offset = plan_bytes(1, 2) + L.total + E.V;
    return RTG_OK;
}

int rtg_golub_kahan(rtg_op op, rtg_sk sk, const float* R0, int m, int basis_dtype, double bd_tol, void* ws,
                    size_t ws_bytes, double* B, double* beta, int* m_done, void* stream) {
    int rc = check_pair(op, sk);
    if (rc) return rc;
    if ((rc = check_m(sk, m))) return rc;
    if (!R0 || !ws || !B || !beta || !m_done) return RTG_E_ARG;
    if (basis_dtype != RTG_F32 && basis_dtype != RTG_BF16) return RTG_E_ARG;
    if (!aligned16(R0) || !aligned16(ws) || !(bd_tol >= 0.0)) return RTG_E_ARG;
    if (sk->identity || !op->adj) return RTG_E_ARG;
    const int bf16 = basis_dtype == RTG_BF16;
    if (ws_bytes < rtg_gk_workspace_bytes(op, sk, m, basis_dtype)) return RTG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const Layout L = problem_layout(op, sk, m, bf16);
    char* base = (char*)ws + plan_bytes(1, 2);
    std::vector<Desc> descs(2);
    fill_desc(descs[0], op, sk, m, bf16, base, L);
    descs[0].R0src = R0;
    descs[0].bd_tol = bd_tol;
    descs[0].keep_last = 1;
    fill_gk_sides(descs[0], descs[1], op, sk, m, bf16, base + L.total);
    Plan plan;
    if ((rc = build_plan(descs, ws, s, plan, 2))) return rc;
    if ((rc = run_gk(plan, 1, m, bf16, false, false, s))) return rc;
    RTG_HIP(launch_finish_arnoldi(plan.d_desc, B, beta, m_done, m, s));
    return RTG_OK;
}

}  // extern "C"

namespace {

// Descriptors and loop bounds of one batch, after the checks of
// rtg_solve_batched.
struct Batch {
    std::vector<Desc> descs;
    int nsides = 1, rmax = 0, mmax = 0, bf16 = 0, skbf = 0;
    bool gk = false, any_x0 = false;
};

int prepare_batch(int count, const rtg_problem* probs, void* ws, size_t ws_bytes, Batch& bt) {
    if (count < 1 || !probs || !ws || !aligned16(ws)) return RTG_E_ARG;
    int basis = -1;
    const int method = probs[0].params.method;
    const bool gk = method == RTG_METHOD_GOLUB_KAHAN;
    for (int p = 0; p < count; ++p) {
        const rtg_problem& q = probs[p];
        int rc = check_pair(q.op, q.sk);
        if (rc) return rc;
        if ((rc = check_m(q.sk, q.params.m))) return rc;
        if ((rc = validate_params(&q.params))) return rc;
        if (q.params.method != method) return RTG_E_ARG;     // one method per batch
        if (gk && (q.sk->identity || !q.op->adj)) return RTG_E_ARG;
        if (!q.C || !q.X || !q.info) return RTG_E_ARG;
        if (!aligned16(q.C) || !aligned16(q.X) || (q.X0 && !aligned16(q.X0))) return RTG_E_ARG;
        if (basis >= 0 && q.params.basis_dtype != basis) return RTG_E_ARG;     // one basis type per batch
        basis = q.params.basis_dtype;
    }
    const int bf16 = basis == RTG_BF16;
    const size_t need = rtg_batch_workspace_bytes(count, probs);
    if (need == 0) return RTG_E_SHAPE;
    if (ws_bytes < need) return RTG_E_WORKSPACE;
    bt.gk = gk;
    bt.bf16 = bf16;
    bt.skbf = basis != RTG_F32;
    bt.nsides = gk ? 2 : 1;
    bt.rmax = 0;
    for (int p = 0; p < count; ++p) bt.rmax = std::max(bt.rmax, probs[p].params.restarts);
    bt.descs.assign((size_t)count * bt.nsides, Desc{});
    size_t off = plan_bytes(count, bt.nsides, bt.rmax > 0);
    bt.mmax = 0;
    bt.any_x0 = false;
    for (int p = 0; p < count; ++p) {
        const rtg_problem& q = probs[p];
        Layout L = problem_layout(q.op, q.sk, q.params.m, bf16);
        char* base = (char*)ws + off;
        Desc& d = bt.descs[p];
        fill_desc(d, q.op, q.sk, q.params.m, bf16, base, L);
        d.skbf = bt.skbf;
        set_params(d, &q.params);
        d.C = q.C;
        d.X0 = q.X0;
        d.X = q.X;
        d.info = q.info;
        d.R0src = q.X0 ? (const void*)d.W : (const void*)q.C;
        off += L.total;
        if (gk) {
            fill_gk_sides(d, bt.descs[(size_t)count + p], q.op, q.sk, q.params.m, bf16, (char*)ws + off);
            off += gk_extra_layout(q.op, q.sk, q.params.m, bf16).total;
        }
        bt.mmax = std::max(bt.mmax, q.params.m);
        bt.any_x0 = bt.any_x0 || q.X0 != nullptr;
    }
    return RTG_OK;
}

// ---- launch shapes per batch shape (the autotuner's table)
struct TuneTable {
    std::mutex mu;
    std::map<std::vector<long long>, rtg_tune> entries;
};

TuneTable& tune_table() {
    static TuneTable t;
    return t;
}

// The shape key of a batch (handles already checked).
std::vector<long long> batch_key(int count, const rtg_problem* probs) {
    std::vector<long long> k{count, probs[0].params.method, probs[0].params.basis_dtype};
    for (int p = 0; p < count; ++p) {
        const rtg_op_s* op = probs[p].op;
        const rtg_sk_s* sk = probs[p].sk;
        const long long row[] = {op->I1, op->I2, op->J, op->r1, op->r2, op->rB, sk->l1, sk->l2, sk->l3,
                                 sk->identity, op->st != nullptr, op->toeplitz, probs[p].params.m,
                                 probs[p].X0 != nullptr};
        k.insert(k.end(), row, row + sizeof(row) / sizeof(row[0]));
    }
    return k;
}

// What a batch can use: slab staging up to slab_cap, Toeplitz taps when
// toep_ok, and where the operator kernel, the fused step and the tile
// kernel's two-row form run at all.
struct TuneCaps {
    int maxJ = 1, slab_cap = 2;
    bool toep_ok = true, stencil = false, phi_runs = true, step_runs = false;
    bool gram_runs = false;   // some problem's Gram chunk follows gram_pairs
    bool persist_ok = false;  // the persistent launch applies (given phi_jt 4 and 16-byte slabs)
};

TuneCaps tune_caps(int count, const rtg_problem* probs) {
    TuneCaps c;
    c.stencil = probs[0].op->st != nullptr;
    bool big = false, bf16 = probs[0].params.basis_dtype == RTG_BF16, step_ok = true, x0 = false;
    bool unsk = probs[0].sk->identity != 0;
    for (int p = 0; p < count; ++p) {
        const rtg_op_s* op = probs[p].op;
        const size_t n = (size_t)op->I1 * op->I2 * op->J;
        c.maxJ = std::max(c.maxJ, op->J);
        big = big || n * 4 > 0x7FFFFFFFull;
        step_ok = step_ok && n * 2 <= 0x7FFFFFFFull && op->a1p[0] != nullptr &&
                  frag_elems(probs[p].sk->l1, op->I1, FRAG_K_BF16) * 4 <= 0x7FFFFFFFull;
        c.toep_ok = c.toep_ok && op->toeplitz;
        x0 = x0 || probs[p].X0 != nullptr;
        const rtg_sk_s* sk = probs[p].sk;
        c.gram_runs = c.gram_runs || (!sk->identity && !gram_split(sk->l3, op->J, (op->I2 + TILE_TC - 1) / TILE_TC));
    }
    c.toep_ok = c.toep_ok && !c.stencil;
    c.slab_cap = big ? 0 : ((c.stencil && c.maxJ <= 3) ? 2 : 1);
    const bool gk = probs[0].params.method == RTG_METHOD_GOLUB_KAHAN;
    c.step_runs = bf16 && step_ok && !c.stencil && !unsk && !gk;
    c.persist_ok = !bf16 && !c.stencil && !unsk && !gk && c.maxJ <= 4 && c.slab_cap >= 1;
    c.phi_runs = !c.step_runs || x0;
    return c;
}

// Every -1 replaced by the default; RTG_E_ARG for a value outside the
// documented set or one the batch cannot use.
int resolve_tune(const TuneCaps& c, const rtg_tune& in, rtg_tune& out) {
    if (in.persist < -1 || in.persist > 1) return RTG_E_ARG;
    if (in.gram_pairs != -1 && in.gram_pairs != 256 && in.gram_pairs != 512 && in.gram_pairs != 1024) return RTG_E_ARG;
    auto one_of = [](int v, int a, int b) { return v == -1 || v == a || v == b; };
    if (!one_of(in.phi_jt, 4, 8) || !one_of(in.tile_rows, 2, 4) || !one_of(in.step_rows, 2, 4)) return RTG_E_ARG;
    if (!one_of(in.phi_toeplitz, 0, 1) || !one_of(in.step_toeplitz, 0, 1)) return RTG_E_ARG;
    if (in.phi_slab < -1 || in.phi_slab > c.slab_cap) return RTG_E_ARG;
    if ((in.phi_toeplitz == 1 || in.step_toeplitz == 1) && !c.toep_ok) return RTG_E_ARG;
    out = rtg_tune{};
    out.phi_jt = in.phi_jt >= 0 ? in.phi_jt : phi_jt(c.maxJ);
    out.phi_slab = in.phi_slab >= 0 ? in.phi_slab : c.slab_cap;
    if (in.phi_toeplitz == 1 && out.phi_slab < 1) return RTG_E_ARG;
    out.phi_toeplitz = in.phi_toeplitz >= 0 ? in.phi_toeplitz : ((c.toep_ok && out.phi_slab >= 1) ? 1 : 0);
    out.tile_rows = in.tile_rows >= 0 ? in.tile_rows : 2;
    out.step_rows = in.step_rows >= 0 ? in.step_rows : 2;
    out.step_toeplitz = in.step_toeplitz >= 0 ? in.step_toeplitz : (c.toep_ok ? 1 : 0);
    out.gram_pairs = in.gram_pairs >= 0 ? in.gram_pairs : GRAM_CH;
    if (in.persist == 1 && (!c.persist_ok || out.phi_jt != 4 || out.phi_slab < 1)) return RTG_E_ARG;
    out.persist = in.persist >= 0 ? in.persist : 0;
    return RTG_OK;
}

rtg_tune tune_unset() {
    rtg_tune t;
    t.phi_jt = t.phi_slab = t.phi_toeplitz = t.tile_rows = t.step_rows = t.step_toeplitz = t.gram_pairs = -1;
    t.persist = -1;
    return t;
}

// the recorded choice for a batch (unset fields when there is none)
rtg_tune lookup_tune(int count, const rtg_problem* probs) {
    const auto key = batch_key(count, probs);
    TuneTable& tt = tune_table();
    std::lock_guard<std::mutex> lock(tt.mu);
    auto it = tt.entries.find(key);
    return it == tt.entries.end() ? tune_unset() : it->second;
}

// The Arnoldi (or Golub-Kahan) loop of a prepared batch, no solve: what the
// autotuner times.
int run_loop(const Plan& plan, const Batch& bt, int count, hipStream_t s) {
    if (bt.gk) return run_gk(plan, count, bt.mmax, bt.bf16, bt.any_x0, false, s);
    return run_solver(plan, count, bt.mmax, bt.bf16, bt.any_x0, false, false, s);
}

// The batched solve; fallback marks every problem's result as the plain
// solver's re-solve (RTG_F_FALLBACK in its flags).
int solve_batched(int count, const rtg_problem* probs, void* ws, size_t ws_bytes, hipStream_t stream,
                  int fallback) {
    Batch bt;
    int rc = prepare_batch(count, probs, ws, ws_bytes, bt);
    if (rc) return rc;
    for (auto& d : bt.descs) d.fallback = fallback;
    hipStream_t s = (hipStream_t)stream;
    rtg_tune tune;
    if ((rc = resolve_tune(tune_caps(count, probs), lookup_tune(count, probs), tune))) return rc;
    Plan plan;
    if ((rc = build_plan(bt.descs, ws, s, plan, bt.nsides, bt.rmax > 0, &tune, true))) return rc;
    if (bt.gk) return run_gk(plan, count, bt.mmax, bt.bf16, bt.any_x0, true, s);
    if ((rc = run_solver(plan, count, bt.mmax, bt.bf16, bt.any_x0, true, false, s))) return rc;
    // restarted RTG-GMRES: every cycle is launched for the whole batch; a
    // problem whose residual is below eps, or whose restarts are spent, sits
    // the cycle out on the device (no host synchronisation)
    for (int c = 1; c <= bt.rmax; ++c)
        if ((rc = run_solver(plan, count, bt.mmax, bt.bf16, true, true, false, s, c))) return rc;
    return RTG_OK;
}

// The plain solver's parameters for the re-solve of a problem: its own mu
// rule and noise level, m steps of RTG-GMRES from X0 = 0 with the given
// basis type, no early stop and no restarts.
rtg_params plain_params(const rtg_params& p, int m, int basis_dtype) {
    rtg_params q = p;
    q.m = m;
    q.basis_dtype = basis_dtype;
    q.stop_res = 0.0;
    q.restarts = 0;
    q.method = RTG_METHOD_GMRES;
    return q;
}

rtg_problem plain_problem(const rtg_problem& p, int m, int basis_dtype) {
    rtg_problem q = p;
    q.X0 = nullptr;
    q.params = plain_params(p.params, m, basis_dtype);
    return q;
}

__global__ void k_gather_flags(const Desc* __restrict__ descs, int count, int* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < count) out[p] = descs[p].info->flags;
}

constexpr int FALLBACK_MASK_ALL = RTG_F_BREAKDOWN | RTG_F_DISCREP_UNREACHABLE | RTG_F_MU_INF | RTG_F_NONFINITE |
                                  RTG_F_NOT_CONVERGED;

// The fallback in two halves.  fallback_begin validates, solves the batch and
// queues the copy of every problem's flags to flags_host (host memory);
// fallback_resolve reads them there and re-solves the failed problems with
// the plain solver, as many at a time as the workspace holds.
int fallback_begin(int count, const rtg_problem* probs, int fb_m, int fb_basis, int fail_mask, void* ws,
                   size_t ws_bytes, int* flags_host, void* stream) {
    if ((fail_mask & ~FALLBACK_MASK_ALL) != 0) return RTG_E_ARG;
    if (fb_basis != RTG_F32 && fb_basis != RTG_BF16) return RTG_E_ARG;
    if (count < 1 || !probs || !ws) return RTG_E_ARG;
    for (int p = 0; p < count; ++p) {
        const rtg_params q = plain_params(probs[p].params, fb_m, fb_basis);
        int rc = validate_params(&q);
        if (rc) return rc;
    }
    const size_t need = rtg_fallback_workspace_bytes(count, probs, fb_m, fb_basis);
    if (need == 0) return RTG_E_SHAPE;
    if (ws_bytes < need) return RTG_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    int rc = solve_batched(count, probs, ws, ws_bytes, s, 0);
    if (rc) return rc;
    // the flags of every problem, gathered through the batch's descriptors
    // (at the start of the workspace) into its last bytes, then copied out
    int* dflags = (int*)((char*)ws + need - align_up((size_t)count * sizeof(int)));
    hipLaunchKernelGGL(k_gather_flags, dim3((count + 255) / 256), dim3(256), 0, s, (const Desc*)ws, count, dflags);
    RTG_HIP(hipGetLastError());
    RTG_HIP(hipMemcpyAsync(flags_host, dflags, (size_t)count * sizeof(int), hipMemcpyDeviceToHost, s));
    return RTG_OK;
}

int fallback_resolve(int count, const rtg_problem* probs, int fb_m, int fb_basis, int fail_mask, void* ws,
                     size_t ws_bytes, const int* flags, int* n_fallback, hipStream_t s) {
    std::vector<rtg_problem> redo;
    for (int p = 0; p < count; ++p)
        if (flags[p] & fail_mask) redo.push_back(plain_problem(probs[p], fb_m, fb_basis));
    *n_fallback = (int)redo.size();
    // re-solve them with the plain solver, as many at a time as the
    // workspace holds (each one alone fits: checked by fallback_begin)
    size_t first = 0;
    while (first < redo.size()) {
        size_t n = 1;
        while (first + n < redo.size() && rtg_batch_workspace_bytes((int)(n + 1), redo.data() + first) <= ws_bytes) ++n;
        int rc = solve_batched((int)n, redo.data() + first, ws, ws_bytes, s, 1);
        if (rc) return rc;
        first += n;
    }
    return RTG_OK;
}

// Events of rtg_solve_batched_fallback_begin, by the host buffer they guard
struct FallbackEvents {
    std::mutex mu;
    std::map<const int*, hipEvent_t> ev;
};
FallbackEvents& fallback_events() {
    static FallbackEvents fe;
    return fe;
}

}  // namespace

extern "C" {

int rtg_solve_batched(int count, const rtg_problem* probs, void* ws, size_t ws_bytes, void* stream) {
    return solve_batched(count, probs, ws, ws_bytes, (hipStream_t)stream, 0);
}

size_t rtg_fallback_workspace_bytes(int count, const rtg_problem* probs, int fb_m, int fb_basis) {
    if (count < 1 || !probs || (fb_basis != RTG_F32 && fb_basis != RTG_BF16)) return 0;
    size_t need = rtg_batch_workspace_bytes(count, probs);
    if (need == 0) return 0;
    for (int p = 0; p < count; ++p) {
        const rtg_problem q = plain_problem(probs[p], fb_m, fb_basis);
        const size_t b = rtg_batch_workspace_bytes(1, &q);
        if (b == 0) return 0;
        need = std::max(need, b);
    }
    return need + align_up((size_t)count * sizeof(int));
}

int rtg_solve_batched_fallback(int count, const rtg_problem* probs, int fb_m, int fb_basis, int fail_mask,
                               void* ws, size_t ws_bytes, int* n_fallback, void* stream) {
    if (!n_fallback) return RTG_E_ARG;
    *n_fallback = 0;
    std::vector<int> flags((size_t)count > 0 ? (size_t)count : 1, 0);
    int rc = fallback_begin(count, probs, fb_m, fb_basis, fail_mask, ws, ws_bytes, flags.data(), stream);
    if (rc) return rc;
    RTG_HIP(hipStreamSynchronize((hipStream_t)stream));
    return fallback_resolve(count, probs, fb_m, fb_basis, fail_mask, ws, ws_bytes, flags.data(), n_fallback,
                            (hipStream_t)stream);
}

int rtg_solve_batched_fallback_begin(int count, const rtg_problem* probs, int fb_m, int fb_basis, int fail_mask,
                                     void* ws, size_t ws_bytes, int* flags_host, void* stream) {
    if (!flags_host) return RTG_E_ARG;
    int rc = fallback_begin(count, probs, fb_m, fb_basis, fail_mask, ws, ws_bytes, flags_host, stream);
    if (rc) return rc;
    hipEvent_t ev = nullptr;
    RTG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    if (hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return RTG_E_HIP;
    }
    FallbackEvents& fe = fallback_events();
    std::lock_guard<std::mutex> lock(fe.mu);
    auto it = fe.ev.find(flags_host);
    if (it != fe.ev.end()) (void)hipEventDestroy(it->second);   // an earlier begin never ended
    fe.ev[flags_host] = ev;
    return RTG_OK;
}

int rtg_solve_batched_fallback_end(int count, const rtg_problem* probs, int fb_m, int fb_basis, int fail_mask,
                                   void* ws, size_t ws_bytes, const int* flags_host, int* n_fallback,
                                   void* stream) {
    if (!n_fallback || !flags_host) return RTG_E_ARG;
    *n_fallback = 0;
    hipEvent_t ev = nullptr;
    {
        FallbackEvents& fe = fallback_events();
        std::lock_guard<std::mutex> lock(fe.mu);
        auto it = fe.ev.find(flags_host);
        if (it == fe.ev.end()) return RTG_E_ARG;                 // no begin for this buffer
        ev = it->second;
        fe.ev.erase(it);
    }
    const hipError_t e = hipEventSynchronize(ev);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return RTG_E_HIP;
    return fallback_resolve(count, probs, fb_m, fb_basis, fail_mask, ws, ws_bytes, flags_host, n_fallback,
                            (hipStream_t)stream);
}

int rtg_tune_set(int count, const rtg_problem* probs, const rtg_tune* tune) {
    if (count < 1 || !probs || !tune) return RTG_E_ARG;
    for (int p = 0; p < count; ++p) {
        int rc = check_pair(probs[p].op, probs[p].sk);
        if (rc) return rc;
    }
    rtg_tune resolved;
    int rc = resolve_tune(tune_caps(count, probs), *tune, resolved);
    if (rc) return rc;
    TuneTable& tt = tune_table();
    std::lock_guard<std::mutex> lock(tt.mu);
    tt.entries[batch_key(count, probs)] = resolved;
    return RTG_OK;
}

int rtg_tune_get(int count, const rtg_problem* probs, rtg_tune* tune) {
    if (count < 1 || !probs || !tune) return RTG_E_ARG;
    for (int p = 0; p < count; ++p) {
        int rc = check_pair(probs[p].op, probs[p].sk);
        if (rc) return rc;
    }
    return resolve_tune(tune_caps(count, probs), lookup_tune(count, probs), *tune);
}

int rtg_set_wait_limit(int polls) {
    if (polls < 0) return RTG_E_ARG;
    g_wait_limit.store(polls);
    return RTG_OK;
}

int rtg_tune_clear(void) {
    TuneTable& tt = tune_table();
    std::lock_guard<std::mutex> lock(tt.mu);
    tt.entries.clear();
    return RTG_OK;
}

int rtg_autotune_batched(int count, const rtg_problem* probs, void* ws, size_t ws_bytes, int reps,
                         rtg_tune* chosen, double* best_ms, void* stream) {
    if (reps < 1 || !chosen) return RTG_E_ARG;
    Batch bt;
    int rc = prepare_batch(count, probs, ws, ws_bytes, bt);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const TuneCaps caps = tune_caps(count, probs);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return RTG_E_HIP;
    }
    // one untimed run (code objects loaded, caches warm), then the minimum
    // over reps timed runs
    auto time_of = [&](const rtg_tune& t, double& ms) -> int {
        std::vector<Desc> descs(bt.descs);
        Plan plan;
        int r = build_plan(descs, ws, s, plan, bt.nsides, false, &t);
        if (r) return r;
        if ((r = run_loop(plan, bt, count, s))) return r;
        ms = std::numeric_limits<double>::infinity();
        for (int k = 0; k < reps; ++k) {
            if (hipEventRecord(e0, s) != hipSuccess) return RTG_E_HIP;
            if ((r = run_loop(plan, bt, count, s))) return r;
            float t_ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess)
                return RTG_E_HIP;
            ms = std::min(ms, (double)t_ms);
        }
        return RTG_OK;
    };
    rtg_tune best;
    double best_t = 0.0;
    rc = resolve_tune(caps, tune_unset(), best);
    if (!rc) rc = time_of(best, best_t);
    // one group of fields at a time, the others at their best so far
    auto try_group = [&](const std::vector<rtg_tune>& cands) -> int {
        for (const rtg_tune& c : cands) {
            double t = 0.0;
            int r = time_of(c, t);
            if (r) return r;
            if (t < best_t) {
                best_t = t;
                best = c;
            }
        }
        return RTG_OK;
    };
    if (!rc && caps.phi_runs) {
        std::vector<rtg_tune> cands;
        for (int jt : {4, 8}) {
            if (jt == 8 && caps.maxJ <= 4) continue;   // half of every tile would be empty
            for (int slab = 0; slab <= caps.slab_cap; ++slab)
                for (int tp = 0; tp <= ((caps.toep_ok && slab >= 1) ? 1 : 0); ++tp) {
                    rtg_tune c = best;
                    c.phi_jt = jt;
                    c.phi_slab = slab;
                    c.phi_toeplitz = tp;
                    cands.push_back(c);
                }
        }
        rc = try_group(cands);
    }
    if (!rc) {
        std::vector<rtg_tune> cands;
        for (int rows : {2, 4}) {
            rtg_tune c = best;
            c.tile_rows = rows;
            cands.push_back(c);
        }
        rc = try_group(cands);
    }
    if (!rc && caps.gram_runs) {
        std::vector<rtg_tune> cands;
        for (int gp : {256, 512, 1024}) {
            rtg_tune c = best;
            c.gram_pairs = gp;
            cands.push_back(c);
        }
        rc = try_group(cands);
    }
    if (!rc && caps.step_runs) {
        std::vector<rtg_tune> cands;
        for (int rows : {2, 4})
            for (int tp = 0; tp <= (caps.toep_ok ? 1 : 0); ++tp) {
                rtg_tune c = best;
                c.step_rows = rows;
                c.step_toeplitz = tp;
                cands.push_back(c);
            }
        rc = try_group(cands);
    }
    // one persistent launch (with the shapes so far, and each Gram chunk:
    // its latency now overlaps other problems' work)
    if (!rc && caps.persist_ok && best.phi_jt == 4 && best.phi_slab >= 1) {
        std::vector<rtg_tune> cands;
        for (int gp : {256, 512, 1024}) {
            if (!caps.gram_runs && gp != best.gram_pairs) continue;
            rtg_tune c = best;
            c.persist = 1;
            c.gram_pairs = caps.gram_runs ? gp : best.gram_pairs;
            cands.push_back(c);
        }
        rc = try_group(cands);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    {
        TuneTable& tt = tune_table();
        std::lock_guard<std::mutex> lock(tt.mu);
        tt.entries[batch_key(count, probs)] = best;
    }
    *chosen = best;
    if (best_ms) *best_ms = best_t;
    return RTG_OK;
}

int rtg_event_timing_enable(int kind_mask) {
    if (kind_mask < 0 || kind_mask >= (1 << NTIMED)) return RTG_E_ARG;
    g_timing.mask = kind_mask;
    return RTG_OK;
}

int rtg_event_timing_read(double* ms, long long* launches, int nkinds) {
    if (nkinds < 0 || (nkinds > 0 && (!ms || !launches))) return RTG_E_ARG;
    int rc = RTG_OK;
    for (int k = 0; k < NTIMED; ++k) {
        double total = 0.0;
        long long cnt = 0;
        for (auto& pr : g_timing.rec[k]) {
            float t = 0.f;
            if (hipEventSynchronize(pr.second) != hipSuccess ||
                hipEventElapsedTime(&t, pr.first, pr.second) != hipSuccess)
                rc = RTG_E_HIP;
            total += t;
            ++cnt;
            g_timing.pool.push_back(pr.first);
            g_timing.pool.push_back(pr.second);
        }
        g_timing.rec[k].clear();
        if (k < nkinds) {
            ms[k] = total;
            launches[k] = cnt;
        }
    }
    return rc;
}

int rtg_solve(rtg_op op, rtg_sk sk, const float* C, const float* X0, const rtg_params* params, void* ws,
              size_t ws_bytes, float* X, rtg_info* info, void* stream) {
    if (!params) return RTG_E_ARG;
    rtg_problem q;
    q.op = op; q.sk = sk; q.C = C; q.X0 = X0; q.X = X; q.params = *params; q.info = info;
    return rtg_solve_batched(1, &q, ws, ws_bytes, stream);
}

}  // extern "C"
