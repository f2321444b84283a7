// lbm_batch.hip -- many independent lattices of uneven sizes advanced by one
// launch per time step (or per two).
//
// The batch state is one caller buffer holding every case's own state
// (same layout as a single lattice, 256-byte aligned, back to back).  A work
// item is one 64 x TY tile of one case; items are numbered case by case and
// a grid of one workgroup per item, or a grid of G workgroups that stride
// over the items (b, b + G, b + 2G, ...), takes them.  Each item runs exactly
// the single-lattice tile body (lbm_fused.hpp) with its case's parameters and
// level stamps, so a case advanced in a batch is bitwise identical to the
// same case advanced alone.  The tile height and G are picked per batch by
// timing the candidates on the batch itself (the autotuner), and K steps are
// captured once into a hipGraph and replayed.
// Batches that hold Cahn-Hilliard or corrected Allen-Cahn cases (the
// two-node-window body of lbm_ch_step.hpp) or local-gradient cases
// (lbm_local_step.hpp) run a second kernel whose LDS holds any of the windows;
// each item runs its case's body.  Batches whose every case runs the plain
// Allen-Cahn step (stencil gradients, present or original model) advance two
// levels per launch, as a single lattice does (lbm_step2.hpp; bitwise two
// one-level steps), with an odd step count ending on a one-level launch.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_ch_step.hpp"
#include "lbm_fused.hpp"
#include "lbm_kernels.hpp"
#include "lbm_local_step.hpp"
#include "lbm_step2.hpp"

namespace lbm {

Layout layout_of(const lbm_params* p);
int validate(const lbm_params* p);
int hip_fail(hipError_t e);
template <typename T>
KParams<T> resolve(const lbm_params* p, const Layout& L);

template <typename T>
struct BatchCase {
    KParams<T> P;
    size_t base;                 // byte offset of the case's state in the batch buffer
    size_t off0, off1, off_stamp;
    int ntx, nty;
    int item_begin;              // first work item of this case
    int body;                    // 0: Allen-Cahn step; 1: Cahn-Hilliard; 2: corrected Allen-Cahn (ACC);
                                 // 3: Allen-Cahn with the local gradient scheme
};

// Case of work item w: the number of cases whose first item is <= w, less
// one.  Every thread of the workgroup tests one case (item_begin ascends with
// the case index) and the workgroup counts the hits: one round of loads
// instead of the dependent loads of a search.
template <typename T>
__device__ __forceinline__ int batch_case(const BatchCase<T>* __restrict__ cases, int ncases, int w, int nthreads) {
    const int tid = threadIdx.y * TX + threadIdx.x;
    int n = 0;
    for (int c0 = 0; c0 < ncases; c0 += nthreads) {
        const int c = c0 + tid;
        n += __syncthreads_count(c < ncases && cases[c].item_begin <= w);
    }
    return n - 1;
}

// NT: non-temporal state stores (the batch's state exceeds the last-level
// cache); ordinary ones otherwise, as for a single lattice.  LOOP: a
// persistent grid (items b, b + G, ...); without it one item per workgroup,
// whose body needs fewer registers (60 against 92 VGPRs for 64 x 4 tiles in
// FP32: 8 waves per SIMD against 5).
template <typename T, int TY, int NBY, bool NT, bool LOOP = true>
__global__ __launch_bounds__(TX* NBY) __attribute__((amdgpu_waves_per_eu(StepWaves<T, TY, NBY>::value)))
void k_step_batch(const BatchCase<T>* __restrict__ cases, int ncases, int nitems, char* batch_state) {
    __shared__ T sphi[TY + 2][TX + 3];
    __shared__ T sphp[TY + 2][TX + 3];
    auto item = [&](int w) {
        const BatchCase<T>& C = cases[batch_case(cases, ncases, w, TX * NBY)];
        const int local = w - C.item_begin;
        // the collision specialisation the case runs alone (lbm_step), so that it stays bitwise
        if (C.P.rates_std)
            step_tile<T, TY, 0, uint32_t, NBY, true, NT>(C.P, batch_state + C.base, C.off0, C.off1, C.off_stamp,
                                                     local % C.ntx, local / C.ntx, nullptr, nullptr, nullptr, sphi, sphp);
        else
            step_tile<T, TY, 0, uint32_t, NBY, false, NT>(C.P, batch_state + C.base, C.off0, C.off1, C.off_stamp,
                                                      local % C.ntx, local / C.ntx, nullptr, nullptr, nullptr, sphi, sphp);
    };
    if constexpr (LOOP) {
        for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
            item(w);
            __syncthreads();   // the next item reuses the LDS window
        }
    } else if ((int)blockIdx.x < nitems) {   // uniform over the workgroup
        item(blockIdx.x);
    }
}

// Two levels per launch: work item blockIdx.x, one 64 x 8 tile of one case, per
// workgroup of 64 x 8 threads (items of a case table for 8-row tiles).  One
// item per workgroup: a loop over items (a persistent grid) doubles the
// registers of the body (169 against 86 VGPRs in FP32).  PER_ITEM: the table
// holds one entry per item (its case's), so that the workgroup reads its case
// directly instead of counting item_begin over the cases first (one round
// trip and a barrier fewer before the tile's loads).
template <typename T, bool NTS, bool PER_ITEM = false>
__global__ __launch_bounds__(TX * 8) void k_step2_batch(const BatchCase<T>* __restrict__ cases, int ncases,
                                                       int nitems, char* batch_state) {
    __shared__ Step2Lds<T, 8> L;
    const int w = blockIdx.x;
    if (w >= nitems) return;   // uniform over the workgroup
    const BatchCase<T>& C = cases[PER_ITEM ? w : batch_case(cases, ncases, w, TX * 8)];
    const int local = w - C.item_begin;
    if (C.P.rates_std)
        step2_tile<T, 8, 8, true, NTS>(C.P, batch_state + C.base, C.off0, C.off1, C.off_stamp, local % C.ntx,
                                       local / C.ntx, L);
    else
        step2_tile<T, 8, 8, false, NTS>(C.P, batch_state + C.base, C.off0, C.off1, C.off_stamp, local % C.ntx,
                                        local / C.ntx, L);
}

// Batches with two-node-window or local-gradient cases: 64 x TY threads (one
// node per thread), the LDS holds any of the windows, each item runs its
// case's body; LOOP as for k_step_batch.
template <typename T, int TY, bool NT, bool LOOP = true>
__global__ __launch_bounds__(TX* TY) void k_step_batch_wide(const BatchCase<T>* __restrict__ cases, int ncases,
                                                            int nitems, char* batch_state) {
    constexpr int NBY = TY;
    __shared__ union {
        struct {
            T sphi[TY + 2][TX + 3];
            T sphp[TY + 2][TX + 3];
        } ac;
        ChWindow<T, TY> ch;
    } lds;
    auto item = [&](int w) {
        const BatchCase<T>& C = cases[batch_case(cases, ncases, w, TX * NBY)];
        const int local = w - C.item_begin;
        const int xt = local % C.ntx, yt = local / C.ntx;
        char* st0 = batch_state + C.base;
        if (C.body == 0 && C.P.rates_std)
            step_tile<T, TY, 0, uint32_t, NBY, true, NT>(C.P, st0, C.off0, C.off1, C.off_stamp, xt, yt, nullptr,
                                                         nullptr, nullptr, lds.ac.sphi, lds.ac.sphp);
        else if (C.body == 0)
            step_tile<T, TY, 0, uint32_t, NBY, false, NT>(C.P, st0, C.off0, C.off1, C.off_stamp, xt, yt, nullptr,
                                                          nullptr, nullptr, lds.ac.sphi, lds.ac.sphp);
        else if (C.body == 1 && C.P.rates_std)
            ch_step_tile<T, TY, 0, false, true, NT, NBY, uint32_t>(C.P, st0, C.off0, C.off1, C.off_stamp, xt, yt,
                                                                   nullptr, nullptr, nullptr, lds.ch);
        else if (C.body == 1)
            ch_step_tile<T, TY, 0, false, false, NT, NBY, uint32_t>(C.P, st0, C.off0, C.off1, C.off_stamp, xt, yt,
                                                                    nullptr, nullptr, nullptr, lds.ch);
        else if (C.body == 3)
            local_step_tile<T, TY, 0, NT, NBY, uint32_t>(C.P, st0, C.off0, C.off1, C.off_stamp, xt, yt, nullptr,
                                                         nullptr, nullptr, lds.ac.sphi);
        else if (C.P.rates_std)
            ch_step_tile<T, TY, 0, true, true, NT, NBY, uint32_t>(C.P, st0, C.off0, C.off1, C.off_stamp, xt, yt,
                                                                  nullptr, nullptr, nullptr, lds.ch);
        else
            ch_step_tile<T, TY, 0, true, false, NT, NBY, uint32_t>(C.P, st0, C.off0, C.off1, C.off_stamp, xt, yt,
                                                                   nullptr, nullptr, nullptr, lds.ch);
    };
    if constexpr (LOOP) {
        for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
            item(w);
            __syncthreads();   // the next item reuses the LDS
        }
    } else if ((int)blockIdx.x < nitems) {   // uniform over the workgroup
        item(blockIdx.x);
    }
}

}  // namespace lbm

using namespace lbm;

// Library-owned plan of a batch: per-case parameters and state offsets, the
// device case table for the chosen tile height, the tuning choice and the
// captured graph.
struct lbm_batch {
    int ncases = 0;
    int dtype = 0;
    std::vector<lbm_params> params;
    std::vector<Layout> layouts;
    std::vector<size_t> base;
    size_t total = 0;
    int autotune = 0;
    bool tuned = false;
    bool wide = false;    // some case runs the two-node-window or local body (one node per thread)
    int ty = 8;
    int by = 4;           // thread rows per workgroup
    int grid = 0;
    int nitems = 0;
    void* d_cases = nullptr;
    int cus = 256;
    // two levels per launch (every case runs the plain Allen-Cahn step), on a
    // case table of 8-row tiles
    bool two_level = false;
    void* d_cases2 = nullptr;
    int nitems2 = 0;
    // graph of `graph_steps` levels for (graph_state, graph_stream)
    hipGraphExec_t graph = nullptr;
    void* graph_state = nullptr;
    hipStream_t graph_stream = nullptr;
    int graph_steps = 0;
};

namespace {

int tiles_for(const lbm_params& p, int ty, int* ntx, int* nty) {
    *ntx = (p.nx + TX - 1) / TX;
    *nty = (p.ny + ty - 1) / ty;
    return *ntx * *nty;
}

// Case table of a batch for tiles of `ty` rows: parameters, state offsets and
// the first work item of every case; returns the number of work items.
template <typename T>
int fill_cases(const lbm_params* params, const Layout* layouts, const size_t* base, int ncases, int ty,
               BatchCase<T>* h) {
    int items = 0;
    for (int c = 0; c < ncases; c++) {
        BatchCase<T>& C = h[c];
        memset(&C, 0, sizeof(C));
        C.P = resolve<T>(&params[c], layouts[c]);
        C.base = base[c];
        C.off0 = layouts[c].off_buf[0];
        C.off1 = layouts[c].off_buf[1];
        C.off_stamp = layouts[c].off_stamp;
        C.item_begin = items;
        const lbm_params& q = params[c];
        C.body = q.phase_eq == LBM_CAHN_HILLIARD ? 1
                 : q.model == LBM_MODEL_CORRECTED ? 2
                 : q.grad_scheme == LBM_GRAD_LOCAL ? 3
                                                   : 0;
        items += tiles_for(params[c], ty, &C.ntx, &C.nty);
    }
    return items;
}

template <typename T>
hipError_t upload_cases(lbm_batch* B, int ty) {
    std::vector<BatchCase<T>> h(B->ncases);
    B->nitems = fill_cases<T>(B->params.data(), B->layouts.data(), B->base.data(), B->ncases, ty, h.data());
    if (!B->d_cases) {
        hipError_t e = hipMalloc(&B->d_cases, sizeof(BatchCase<T>) * B->ncases);
        if (e != hipSuccess) return e;
    }
    return hipMemcpy(B->d_cases, h.data(), sizeof(BatchCase<T>) * B->ncases, hipMemcpyHostToDevice);
}

// The case table of the two-level launch (8-row tiles).
template <typename T>
hipError_t upload_cases2(lbm_batch* B) {
    std::vector<BatchCase<T>> h(B->ncases);
    B->nitems2 = fill_cases<T>(B->params.data(), B->layouts.data(), B->base.data(), B->ncases, 8, h.data());
    // one entry per item: entry w is the case of item w (k_step2_batch, PER_ITEM)
    std::vector<BatchCase<T>> items((size_t)B->nitems2);
    for (int c = 0; c < B->ncases; c++) {
        const int end = c + 1 < B->ncases ? h[c + 1].item_begin : B->nitems2;
        for (int w = h[c].item_begin; w < end; w++) items[(size_t)w] = h[c];
    }
    hipError_t e = hipMalloc(&B->d_cases2, sizeof(BatchCase<T>) * items.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(B->d_cases2, items.data(), sizeof(BatchCase<T>) * items.size(), hipMemcpyHostToDevice);
}

// One launch of the batch kernels over `nitems` work items of a device case
// table (grid 0: one workgroup per item).
struct BatchShape {
    int ty, by, grid, nitems, ncases;
    bool wide;
    size_t total;   // bytes of the batch state (store policy)
};

template <typename T, int TY, int NBY>
void batch_launch(const BatchShape& S, const void* d_cases, char* state, hipStream_t s) {
    const BatchCase<T>* cases = reinterpret_cast<const BatchCase<T>*>(d_cases);
    const bool nt = S.total > (size_t)LBM_NT_MIN_BYTES;
    if (S.grid > 0 && S.grid < S.nitems) {
        if (nt) k_step_batch<T, TY, NBY, true><<<S.grid, dim3(TX, NBY), 0, s>>>(cases, S.ncases, S.nitems, state);
        else k_step_batch<T, TY, NBY, false><<<S.grid, dim3(TX, NBY), 0, s>>>(cases, S.ncases, S.nitems, state);
    } else {
        if (nt) k_step_batch<T, TY, NBY, true, false><<<S.nitems, dim3(TX, NBY), 0, s>>>(cases, S.ncases, S.nitems, state);
        else k_step_batch<T, TY, NBY, false, false><<<S.nitems, dim3(TX, NBY), 0, s>>>(cases, S.ncases, S.nitems, state);
    }
}

template <typename T, int TY>
void batch_launch_wide(const BatchShape& S, const void* d_cases, char* state, hipStream_t s) {
    const BatchCase<T>* cases = reinterpret_cast<const BatchCase<T>*>(d_cases);
    const bool nt = S.total > (size_t)LBM_NT_MIN_BYTES;
    const dim3 blk(TX, TY);
    if (S.grid > 0 && S.grid < S.nitems) {
        if (nt) k_step_batch_wide<T, TY, true><<<S.grid, blk, 0, s>>>(cases, S.ncases, S.nitems, state);
        else k_step_batch_wide<T, TY, false><<<S.grid, blk, 0, s>>>(cases, S.ncases, S.nitems, state);
    } else {
        if (nt) k_step_batch_wide<T, TY, true, false><<<S.nitems, blk, 0, s>>>(cases, S.ncases, S.nitems, state);
        else k_step_batch_wide<T, TY, false, false><<<S.nitems, blk, 0, s>>>(cases, S.ncases, S.nitems, state);
    }
}

template <typename T>
void launch_batch_shape(const BatchShape& S, const void* d_cases, char* state, hipStream_t s) {
    constexpr int T16 = sizeof(T) == 8 ? 8 : 16;
    if (S.wide) {
        if (S.ty == 4) batch_launch_wide<T, 4>(S, d_cases, state, s);
        else batch_launch_wide<T, 8>(S, d_cases, state, s);
        return;
    }
    if (S.ty == 4) batch_launch<T, 4, 4>(S, d_cases, state, s);
    else if (S.ty == 8 || sizeof(T) == 8) {
        if (S.by == 8) batch_launch<T, 8, 8>(S, d_cases, state, s);
        else batch_launch<T, 8, 4>(S, d_cases, state, s);
    } else {
        if (S.by == 8) batch_launch<T, T16, 8>(S, d_cases, state, s);
        else batch_launch<T, T16, 4>(S, d_cases, state, s);
    }
}

template <typename T>
void launch_batch_once(lbm_batch* B, char* state, hipStream_t s) {
    const BatchShape S{B->ty, B->by, B->grid, B->nitems, B->ncases, B->wide, B->total};
    launch_batch_shape<T>(S, B->d_cases, state, s);
}

// One two-level launch over `nitems` items of a case table for 8-row tiles
// (per_item: one entry per item, as upload_cases2 writes it; else one per case).
template <typename T>
void launch_batch2(int nitems, int ncases, const void* d_cases, size_t total, char* state, hipStream_t s,
                   bool per_item) {
    const BatchCase<T>* cases = reinterpret_cast<const BatchCase<T>*>(d_cases);
    const bool nts = total > (size_t)LBM_NT_MIN_BYTES;
    if (per_item) {
        if (nts) k_step2_batch<T, true, true><<<nitems, dim3(TX, 8), 0, s>>>(cases, ncases, nitems, state);
        else k_step2_batch<T, false, true><<<nitems, dim3(TX, 8), 0, s>>>(cases, ncases, nitems, state);
    } else {
        if (nts) k_step2_batch<T, true><<<nitems, dim3(TX, 8), 0, s>>>(cases, ncases, nitems, state);
        else k_step2_batch<T, false><<<nitems, dim3(TX, 8), 0, s>>>(cases, ncases, nitems, state);
    }
}

// `n` levels of the batch: two-level launches, and a one-level launch for an odd n.
template <typename T>
void launch_batch_levels(lbm_batch* B, char* state, int64_t n, hipStream_t s) {
    if (B->two_level) {
        for (int64_t t = 0; t + 2 <= n; t += 2)
            launch_batch2<T>(B->nitems2, B->ncases, B->d_cases2, B->total, state, s, true);
        if (n & 1) launch_batch_once<T>(B, state, s);
    } else {
        for (int64_t t = 0; t < n; t++) launch_batch_once<T>(B, state, s);
    }
}

void drop_graph(lbm_batch* B) {
    if (B->graph) (void)hipGraphExecDestroy(B->graph);
    B->graph = nullptr;
    B->graph_state = nullptr;
    B->graph_stream = nullptr;
    B->graph_steps = 0;
}

template <typename T>
int batch_step_t(lbm_batch* B, char* state, int64_t nsteps, hipStream_t s) {
    constexpr int K = 32;   // steps per captured graph
    hipError_t e;
    // not while the caller captures the stream: the launches go into its graph
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s != nullptr && nsteps >= K) {
        e = hipStreamIsCapturing(s, &cs);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (s != nullptr && nsteps >= K && cs == hipStreamCaptureStatusNone) {
        if (!B->graph || B->graph_state != state || B->graph_stream != s) {
            drop_graph(B);
            hipGraph_t g;
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e);
            launch_batch_levels<T>(B, state, K, s);
            e = hipStreamEndCapture(s, &g);
            if (e != hipSuccess) return hip_fail(e);
            e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(e);
            B->graph_state = state;
            B->graph_stream = s;
            B->graph_steps = K;
        }
        for (int64_t t = 0; t + K <= nsteps; t += K) {
            e = hipGraphLaunch(B->graph, s);
            if (e != hipSuccess) return hip_fail(e);
        }
        nsteps %= K;
    }
    launch_batch_levels<T>(B, state, nsteps, s);
    e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

template <typename T>
int batch_init_cases(lbm_batch* B, char* state, const void* const* phi0, const void* const* p0, hipStream_t s) {
    for (int c = 0; c < B->ncases; c++) {
        int rc = lbm_init(&B->params[c], state + B->base[c], phi0[c], nullptr, p0 ? p0[c] : nullptr, s);
        if (rc) return rc;
    }
    return LBM_OK;
}

// Time every candidate (tile height, persistent grid) on the batch itself and
// keep the fastest; the state is re-initialised afterwards by the caller.
template <typename T>
int autotune_t(lbm_batch* B, char* state, const void* const* phi0, const void* const* p0, hipStream_t s) {
    const int shapes[5][2] = {{4, 4}, {8, 4}, {8, 8}, {16, 4}, {16, 8}};   // (tile rows, thread rows)
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LBM_E_HIP;
    float best = 1e30f;
    int best_ty = 8, best_by = 4, best_grid = 0;
    for (const auto& sh : shapes) {
        const int ty = sh[0];
        if (ty == 16 && sizeof(T) == 8) continue;
        if (B->wide && (sh[1] != ty || ty > 8)) continue;   // the wide bodies: one node per thread
        B->ty = ty;
        B->by = sh[1];
        hipError_t e = upload_cases<T>(B, ty);
        if (e != hipSuccess) return hip_fail(e);
        const int grids[4] = {0, 2 * B->cus, 4 * B->cus, 8 * B->cus};
        for (int g : grids) {
            if (g > B->nitems) continue;
            B->grid = g;
            int rc = batch_init_cases<T>(B, state, phi0, p0, s);
            if (rc) return rc;
            for (int w = 0; w < 3; w++) launch_batch_once<T>(B, state, s);
            (void)hipEventRecord(e0, s);
            for (int w = 0; w < 10; w++) launch_batch_once<T>(B, state, s);
            (void)hipEventRecord(e1, s);
            e = hipEventSynchronize(e1);
            if (e != hipSuccess) return hip_fail(e);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) {
                best = ms;
                best_ty = ty;
                best_by = sh[1];
                best_grid = g;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    B->ty = best_ty;
    B->by = best_by;
    B->grid = best_grid;
    hipError_t e = upload_cases<T>(B, best_ty);
    if (e != hipSuccess) return hip_fail(e);
    B->tuned = true;
    return LBM_OK;
}

// Every case valid, one dtype, each case's state copy addressable with 32-bit offsets.
int validate_batch(const lbm_params* cases, int ncases) {
    if (ncases < 1) return LBM_E_SIZE;
    for (int c = 0; c < ncases; c++) {
        int rc = validate(&cases[c]);
        if (rc) return rc;
        if (cases[c].dtype != cases[0].dtype) return LBM_E_DTYPE;
        Layout L = layout_of(&cases[c]);
        if (L.buf_bytes >= (size_t(1) << 32)) return LBM_E_SIZE;   // 32-bit offsets within a case
    }
    return LBM_OK;
}

// Byte offset of every case's state in a batch state (each rounded up to 256 B);
// returns the total.
size_t batch_offsets(const lbm_params* cases, int ncases, Layout* layouts, size_t* base) {
    size_t off = 0;
    for (int c = 0; c < ncases; c++) {
        layouts[c] = layout_of(&cases[c]);
        base[c] = off;
        off += (layouts[c].total + 255) / 256 * 256;
    }
    return off;
}

bool wide_batch(const lbm_params* cases, int ncases) {
    bool w = false;
    for (int c = 0; c < ncases; c++)
        w = w || cases[c].phase_eq == LBM_CAHN_HILLIARD || cases[c].model == LBM_MODEL_CORRECTED ||
            cases[c].grad_scheme == LBM_GRAD_LOCAL;
    return w;
}

// Two levels per launch: every case runs the plain Allen-Cahn step (stencil
// gradients, present or original model) and the batch has at least 256 tiles
// of 64 x 8 nodes, the size rule of a single lattice (lbm_step.hip).  The
// environment variable LBM_TWO_LEVEL, read when a plan is made (and at every
// call of the allocation-free step), overrides the size rule: "0" never, "1"
// whatever the size.
bool two_level_batch(const lbm_params* cases, int ncases) {
    long long tiles8 = 0;
    for (int c = 0; c < ncases; c++) {
        const lbm_params& q = cases[c];
        if (q.phase_eq != LBM_ALLEN_CAHN || q.model == LBM_MODEL_CORRECTED || q.grad_scheme != LBM_GRAD_STENCIL)
            return false;
        int ntx, nty;
        tiles8 += tiles_for(q, 8, &ntx, &nty);
    }
    const char* e = getenv("LBM_TWO_LEVEL");
    if (e && e[0] == '0' && e[1] == 0) return false;
    if (e && e[0] == '1' && e[1] == 0) return true;
    return tiles8 >= 256;
}

// ---- the batch step that allocates nothing (lbm_batch_step_noalloc) ----
// Its case table lives in `scratch`, a fixed array of the library in every
// GPU's memory.  In host code `scratch` only names the symbol: the kernels get
// the device address that hipGetSymbolAddress returns for the current device
// (looked up once per device, on the first call there).
constexpr size_t NOALLOC_CASE_BYTES =
    sizeof(BatchCase<double>) > sizeof(BatchCase<float>) ? sizeof(BatchCase<double>) : sizeof(BatchCase<float>);
static_assert(LBM_NOALLOC_MAX_CASES * NOALLOC_CASE_BYTES <= (size_t(256) << 10), "case table above 256 KB");
static __device__ __align__(256) unsigned char scratch[LBM_NOALLOC_MAX_CASES * NOALLOC_CASE_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;   // device address of `scratch`, per device ordinal

hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)dev >= g_scratch_dev.size()) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// A few cases of the table travel in the kernel arguments (copied at launch,
// so the host table may go away as soon as the launch returns) and are stored
// into the device table by one small workgroup.
template <typename T>
struct CaseChunk {
    static constexpr int N = (int)(3072 / sizeof(BatchCase<T>)) > 0 ? (int)(3072 / sizeof(BatchCase<T>)) : 1;
    BatchCase<T> c[N];
    int first, count;
};

template <typename T>
__global__ void k_put_cases(CaseChunk<T> chunk, BatchCase<T>* dst) {
    for (int i = threadIdx.x; i < chunk.count; i += blockDim.x) dst[chunk.first + i] = chunk.c[i];
}

template <typename T>
int batch_step_noalloc_t(const lbm_params* cases, int ncases, char* state, int64_t nsteps, hipStream_t s) {
    // host-side tables on the stack: at most LBM_NOALLOC_MAX_CASES cases
    static_assert(LBM_NOALLOC_MAX_CASES <= 256, "stack tables");
    Layout layouts[LBM_NOALLOC_MAX_CASES];
    size_t base[LBM_NOALLOC_MAX_CASES];
    const size_t total = batch_offsets(cases, ncases, layouts, base);
    void* dtab = nullptr;
    hipError_t e = scratch_address(&dtab);
    if (e != hipSuccess) return hip_fail(e);
    BatchCase<T>* table = reinterpret_cast<BatchCase<T>*>(dtab);
    // the untuned plan's shape: 8-row tiles, 64 x 4 threads (64 x 8 for the wide bodies), one
    // workgroup per item; the same table serves the two-level launch (8-row tiles too)
    const int ty = 8;
    CaseChunk<T> chunk;
    int nitems = 0;
    for (int c0 = 0; c0 < ncases; c0 += CaseChunk<T>::N) {
        const int cnt = ncases - c0 < CaseChunk<T>::N ? ncases - c0 : CaseChunk<T>::N;
        memset(&chunk, 0, sizeof(chunk));
        const int items = fill_cases<T>(cases + c0, layouts + c0, base + c0, cnt, ty, chunk.c);
        for (int i = 0; i < cnt; i++) chunk.c[i].item_begin += nitems;
        nitems += items;
        chunk.first = c0;
        chunk.count = cnt;
        k_put_cases<T><<<1, 64, 0, s>>>(chunk, table);
    }
    const bool wide = wide_batch(cases, ncases);
    const BatchShape S{ty, wide ? ty : 4, 0, nitems, ncases, wide, total};
    int64_t t = 0;
    if (two_level_batch(cases, ncases))
        for (; t + 2 <= nsteps; t += 2) launch_batch2<T>(nitems, ncases, table, total, state, s, false);
    for (; t < nsteps; t++) launch_batch_shape<T>(S, table, state, s);
    e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}

}  // namespace

extern "C" {

int lbm_batch_create(const lbm_params* cases, int32_t ncases, int32_t autotune, lbm_batch** out) {
    if (!cases || !out) return LBM_E_NULL;
    int rc = validate_batch(cases, ncases);
    if (rc) return rc;
    lbm_batch* B = new lbm_batch();
    B->ncases = ncases;
    B->dtype = cases[0].dtype;
    B->autotune = autotune;
    B->params.assign(cases, cases + ncases);
    B->wide = wide_batch(cases, ncases);
    B->layouts.resize(ncases);
    B->base.resize(ncases);
    B->total = batch_offsets(cases, ncases, B->layouts.data(), B->base.data());
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&B->cus, hipDeviceAttributeMultiprocessorCount, dev);
    // default (untuned) choice: 8-row tiles, one workgroup per item (64 x 4 threads; the
    // wide bodies: 64 x 8, one node per thread)
    B->ty = 8;
    B->by = B->wide ? 8 : 4;
    B->grid = 0;
    // LBM_BATCH_SHAPE="ty,by,grid" fixes the one-level shape (no autotuning):
    // one of the tuner's candidates, grid 0 for one workgroup per item
    if (const char* env = getenv("LBM_BATCH_SHAPE")) {
        int ty = 0, by = 0, grid = -1;
        const bool ok = sscanf(env, "%d,%d,%d", &ty, &by, &grid) == 3 && grid >= 0 &&
                        ((ty == 4 && by == 4) || ((ty == 8 || ty == 16) && (by == 4 || by == 8))) &&
                        !(ty == 16 && B->dtype == LBM_F64) && !(B->wide && (by != ty || ty > 8));
        if (!ok) {
            delete B;
            return LBM_E_PARAM;
        }
        B->ty = ty;
        B->by = by;
        B->grid = grid;
        B->tuned = true;
    }
    hipError_t e = B->dtype == LBM_F32 ? upload_cases<float>(B, B->ty) : upload_cases<double>(B, B->ty);
    B->two_level = two_level_batch(cases, ncases);
    if (e == hipSuccess && B->two_level) e = B->dtype == LBM_F32 ? upload_cases2<float>(B) : upload_cases2<double>(B);
    if (e != hipSuccess) {
        lbm_batch_destroy(B);
        return hip_fail(e);
    }
    *out = B;
    return LBM_OK;
}

int lbm_batch_state_size(const lbm_batch* B, size_t* nbytes) {
    if (!B || !nbytes) return LBM_E_NULL;
    *nbytes = B->total;
    return LBM_OK;
}

int lbm_batch_case_offset(const lbm_batch* B, int32_t c, size_t* offset) {
    if (!B || !offset) return LBM_E_NULL;
    if (c < 0 || c >= B->ncases) return LBM_E_SIZE;
    *offset = B->base[c];
    return LBM_OK;
}

int lbm_batch_init(lbm_batch* B, void* state, const void* const* phi0, const void* const* p0, void* stream) {
    if (!B || !state || !phi0) return LBM_E_NULL;
    if ((uintptr_t)state % 256) return LBM_E_SIZE;
    for (int c = 0; c < B->ncases; c++)
        if (!phi0[c]) return LBM_E_NULL;
    hipStream_t s = (hipStream_t)stream;
    drop_graph(B);
    if (B->autotune && !B->tuned) {
        int rc = B->dtype == LBM_F32 ? autotune_t<float>(B, (char*)state, phi0, p0, s)
                                     : autotune_t<double>(B, (char*)state, phi0, p0, s);
        if (rc) return rc;
    }
    return B->dtype == LBM_F32 ? batch_init_cases<float>(B, (char*)state, phi0, p0, s)
                               : batch_init_cases<double>(B, (char*)state, phi0, p0, s);
}

int lbm_batch_step(lbm_batch* B, void* state, int64_t nsteps, void* stream) {
    if (!B || !state) return LBM_E_NULL;
    if (nsteps < 0) return LBM_E_SIZE;
    hipStream_t s = (hipStream_t)stream;
    return B->dtype == LBM_F32 ? batch_step_t<float>(B, (char*)state, nsteps, s)
                               : batch_step_t<double>(B, (char*)state, nsteps, s);
}

int lbm_batch_step_noalloc(const lbm_params* cases, int32_t ncases, void* state, int64_t nsteps, void* stream) {
    if (!cases || !state) return LBM_E_NULL;
    if (ncases > LBM_NOALLOC_MAX_CASES) return LBM_E_SIZE;
    int rc = validate_batch(cases, ncases);
    if (rc) return rc;
    if (nsteps < 0) return LBM_E_SIZE;
    if ((uintptr_t)state % 256) return LBM_E_SIZE;
    if (nsteps == 0) return LBM_OK;
    hipStream_t s = (hipStream_t)stream;
    return cases[0].dtype == LBM_F32 ? batch_step_noalloc_t<float>(cases, ncases, (char*)state, nsteps, s)
                                     : batch_step_noalloc_t<double>(cases, ncases, (char*)state, nsteps, s);
}

int lbm_batch_tuning(const lbm_batch* B, int32_t* tile_rows, int32_t* thread_rows, int32_t* grid, int32_t* items) {
    if (!B) return LBM_E_NULL;
    if (tile_rows) *tile_rows = B->ty;
    if (thread_rows) *thread_rows = B->by;
    if (grid) *grid = B->grid > 0 ? B->grid : B->nitems;
    if (items) *items = B->nitems;
    return LBM_OK;
}

int lbm_batch_levels_per_launch(const lbm_batch* B, int32_t* levels) {
    if (!B || !levels) return LBM_E_NULL;
    *levels = B->two_level ? 2 : 1;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* B) {
    if (!B) return LBM_E_NULL;
    drop_graph(B);
    if (B->d_cases) (void)hipFree(B->d_cases);
    if (B->d_cases2) (void)hipFree(B->d_cases2);
    delete B;
    return LBM_OK;
}

}  // extern "C"
