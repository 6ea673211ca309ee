// libtrafficsim: the traffic microsimulation step of Waddell et al., Sec. 6,
// as hand-written HIP for CDNA4 (gfx950).
//
// One synchronous step t -> t+1 (every decision reads state t only):
//   k_decide   first blocks, per departure queue (Sec. 6.2.2): release the
//              trips due now, entry-lane choice, the head's entry claim.
//              Other blocks, per vehicle: leader search, IDM acceleration
//              (Sec. 6.3.2, car-following equation), ballistic update,
//              link-end crossing (claim) or arrival (Sec. 6.3.1 routes);
//              then, in the same thread, for a vehicle that may change
//              lanes: candidates, gap acceptance, safety and incentive
//              (Sec. 6.3.2 lane changing); the best candidate claims.  The
//              block's tile of the sorted arrays sits in LDS, so the vehicles
//              around a vehicle, in its lane and the neighbouring ones, are
//              mostly LDS reads.  Claims take one-metre cells of their target
//              lane with a 64-bit atomicMin of (epoch, vehicle id).
//   k_resolve  per claim: it wins iff it still owns all its cells (no
//              overlapping claim with a lower id); winners find their gap in
//              the sorted order and take a slot in it.
//   k_scan     exclusive scan (decoupled look-back) of stay[i] + movers-in-gap[i]
//              gives every survivor and every gap its new position.
//   k_scatter  survivors write their record to the new buffer; movers stage
//              their (lane, x) keys per gap.
//   k_place    movers rank themselves inside their gap and write their
//              record.
//   k_lanes    index the lanes of the new buffer; commit the step's counters.
//
// Vehicle state is structure-of-arrays, double-buffered, kept sorted by
// (global lane id, position), so the vehicle ahead in the lane is the next
// array element (coalesced) and the run of any lane is one read of the lane
// index.  The whole loop runs without host round trips.
//
// Floating point: built with -ffp-contract=off; every expression below is
// evaluated in float in the order written (correctly rounded divide), so a
// CPU float implementation of the same rules reproduces it bit for bit.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "trafficsim.h"

#include "common.h"
#include "step_kernels.h"
#include "adjoint_kernels.h"
#include "check_kernels.h"

using namespace tsim;


// ===========================================================================
// host side
// ===========================================================================

// a trip state (the arrays of Trips that change as vehicles enter links)
struct Cold {
    int* rcur = nullptr;
    int* kin = nullptr;
    float* phin = nullptr;
};

static Cold cold_of(const Trips& t) {
    Cold c;
    c.rcur = t.rcur;
    c.kin = t.kin;
    c.phin = t.phin;
    return c;
}

struct sim_t {
    hipStream_t stream = nullptr;
    sim_alloc_fn alloc = nullptr;
    sim_free_fn free_fn = nullptr;
    void* ctx = nullptr;
    std::string err;
    std::vector<void*> allocs;

    int nn = 0, ne = 0, nlanes = 0, ncls = 0;
    std::vector<int> row_ptr, col_idx, lanes, cls, lane_base, ncell, tail;
    // vehicle types (Sec. 6.3.5): acceleration and speed caps per type, the
    // car-following inputs the per-type constants derive from, trip types
    std::vector<double> tamax{INFINITY}, tvmax{INFINITY};
    std::vector<float> idm_in;
    std::vector<unsigned char> trip_type;
    bool typed = false;
    DrvRec* d_drv = nullptr;
    unsigned char* d_capA = nullptr;
    unsigned char* d_capV = nullptr;
    unsigned char* d_vtype = nullptr;
    std::vector<float> len, speed;
    long long ncells = 0;

    Params P{};
    Net net{};
    Trips tr{};
    Veh buf[2]{};
    Scratch s{};
    int* qstate = nullptr;  // departure queues: heads [0, nq), then tails [nq, 2 nq)
    Counters* ctr = nullptr;
    float* d_inv_v0 = nullptr;
    float* d_cT = nullptr;
    float* d_cA = nullptr;
    float* d_cKab = nullptr;
    float* d_cVs = nullptr;
    float* d_cB = nullptr;
    unsigned* d_epoch = nullptr;
    GridSync* d_gsync = nullptr;  // the persistent step's barrier state
    int persist_res[2] = {0, 0};  // resident blocks of k_steps<1>, k_steps<2> on the device (0 unknown)
    // intersection control: per node kind, per edge inbound rank, per node inbound degree
    int* d_ctrl = nullptr;
    int* d_in_rank = nullptr;
    int* d_in_deg = nullptr;
    int* d_rholder = nullptr;  // stop-node holders of the recompute pass

    bool loaded = false;
    int cap = 0;
    int ntrips = 0;
    // what a route reload needs of the demand: its first step, whether it
    // placed vehicles, per vehicle id the trip index and departure step, the
    // capacities of the route table and of the departure queues
    long long t_load = 0;
    bool placed = false;
    int* d_ord = nullptr;
    int* d_dep = nullptr;
    long long re_cap = 0;
    int nq_cap = 0;
    // route reload scratch (allocated at the first reload)
    int* d_tail = nullptr;
    unsigned* d_rkey = nullptr;  // [2 x cap] queue keys, then sorted
    int* d_rval = nullptr;       // [2 x cap] vehicle ids, then queue flags and indices
    int* d_rerr = nullptr;       // [2] first bad route, queue count
    void* d_rtmp = nullptr;
    size_t rtmp_bytes = 0;
    // state check (allocated at the first check): a bit per vehicle id, the
    // count and the lowest offending entry per class
    unsigned* d_chk_seen = nullptr;
    unsigned long long* d_chk_fail = nullptr;
    int* d_chk_first = nullptr;
    long long host_t = 0;  // steps enqueued so far (selects the buffer parity)
    int grid = 1;
    int grid_small = 1;  // k_scan's persistent blocks
    int grid_q = 1;      // k_decide's departure-queue blocks: one thread per queue
    int dshape = 0;      // k_decide's launch shape (kDecideShapes)
    std::vector<int> h_rbeg;
    int timing_every = 0;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::vector<hipEvent_t>> ev_steps;  // a start and a stop event per kernel of a sampled step

    // differentiation window: checkpoints every `tape_every` steps from tape_t0
    struct Ckpt {
        long long t = 0;
        Veh v{};
        Cold c{};
        int* qstate = nullptr;
        Counters* ctr = nullptr;
        int* holder = nullptr;
    };
    bool tape_on = false;
    long long tape_t0 = 0;
    int tape_every = 0;
    size_t nckpt = 0;
    std::vector<Ckpt> ckpt_pool;
    // recompute state and adjoint work arrays (allocated at the first sim_grad)
    bool adj_ready = false;
    long long tape_full_t = -1;  // the tape slices hold the whole window [tape_t0, tape_full_t)
    double* d_rF = nullptr;      // replay: per-link sums of the traversals' fraction differences
    double* d_r64 = nullptr;     // FP64 replay: state (two buffers of x, v) and entry fractions, 5 x cap
    double* d_r64c = nullptr;    // FP64 replay: its IDM constants
    Veh rbuf[2]{};
    Cold rcold{};            // trip state of the recompute pass
    int* rqstate = nullptr;  // queue heads and tails of the recompute pass
    Counters* rctr = nullptr;
    Tape slab{};  // tape_every slices of cap entries
    AdjState adj{};
    float *L0x = nullptr, *L0v = nullptr, *L1x = nullptr, *L1v = nullptr;
    unsigned long long* sink = nullptr;  // statistics of the recompute pass (discarded)
    int adj_grid = 0;
    int adj_k = 0;  // tape slices allocated

    // batch of scenarios: edge offset of each scenario (size n+1), empty otherwise
    std::vector<int> batch_edge_off;
    // captured multi-step graphs, by (parity of the first step, chunk length)
    struct GraphEntry {
        int parity = 0, chunk = 0;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphEntry> graphs;
    // graphs are captured and replayed on a stream of the library's own (the
    // caller's stream may be the legacy default stream, which cannot be
    // captured), ordered after and before the caller's work by two events
    hipStream_t gstream = nullptr;
    hipEvent_t gjoin[2] = {nullptr, nullptr};
};

namespace {

int fail(sim_t* S, int code, const std::string& msg) {
    if (S) S->err = msg;
    return code;
}

// a failed call also clears the thread's last-error state, so that it is not
// reported again by the caller's next, unrelated HIP call
#define HIPCHECK(S, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (void)hipGetLastError();                                                             \
            return fail((S), SIM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));        \
        }                                                                                        \
    } while (0)

void* raw_alloc(sim_t* S, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (S->alloc) {
        p = S->alloc(S->ctx, bytes);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) S->allocs.push_back(p);
    return p;
}

template <class T>
bool dalloc(sim_t* S, T*& out, size_t n) {
    out = static_cast<T*>(raw_alloc(S, sizeof(T) * (n ? n : 1)));
    return out != nullptr;
}

// frees one allocation of the handle (after the stream has drained)
template <class T>
void dfree(sim_t* S, T*& p) {
    if (!p) return;
    void* raw = const_cast<void*>(static_cast<const void*>(p));
    auto it = std::find(S->allocs.begin(), S->allocs.end(), raw);
    if (it != S->allocs.end()) {
        (void)hipStreamSynchronize(S->stream);
        if (S->free_fn) S->free_fn(S->ctx, raw);
        else (void)hipFree(raw);
        S->allocs.erase(it);
    }
    p = nullptr;
}

void release_all(sim_t* S) {
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    else (void)hipDeviceSynchronize();
    for (void* p : S->allocs) {
        if (S->free_fn) S->free_fn(S->ctx, p);
        else (void)hipFree(p);
    }
    S->allocs.clear();
}

// Per (class, type) and (link, type) constants in double, rounded once: a
// type caps the class's maximum acceleration and the link's desired speed
// (Sec. 6.3.5); with no cap (infinite) they are the class's own values.
int upload_idm(sim_t* S, const float* idm) {
    const int nt = S->P.nt, nc = S->ncls;
    std::vector<float> T(nc), A((size_t)nc * nt), K((size_t)nc * nt), VS(nc), B(nc), inv((size_t)S->ne * nt);
    std::vector<unsigned char> capA((size_t)nc * nt), capV((size_t)S->ne * nt);
    for (int c = 0; c < nc; ++c) {
        double s0 = idm[4 * c + 0], t = idm[4 * c + 1], a = idm[4 * c + 2], b = idm[4 * c + 3];
        if (!(s0 > 0) || !(t >= 0) || !(a > 0) || !(b > 0) || !std::isfinite(s0 * t * a * b))
            return fail(S, SIM_EINVAL, "idm parameters of class " + std::to_string(c) + " out of range");
        T[c] = (float)t;
        VS[c] = (float)s0;
        B[c] = (float)b;
        for (int k = 0; k < nt; ++k) {
            const double ak = a < S->tamax[k] ? a : S->tamax[k];
            A[(size_t)c * nt + k] = (float)ak;
            K[(size_t)c * nt + k] = (float)(1.0 / (2.0 * std::sqrt(ak * b)));
            capA[(size_t)c * nt + k] = !(a < S->tamax[k]);
        }
    }
    for (int e = 0; e < S->ne; ++e) {
        const double v0 = (double)idm[4 * S->cls[e] + 0] * (double)S->speed[e];
        for (int k = 0; k < nt; ++k) {
            inv[(size_t)e * nt + k] = (float)(1.0 / (v0 < S->tvmax[k] ? v0 : S->tvmax[k]));
            capV[(size_t)e * nt + k] = !(v0 < S->tvmax[k]);
        }
    }
    S->idm_in.assign(idm, idm + 4 * (size_t)nc);
    const hipMemcpyKind h = hipMemcpyHostToDevice;
    HIPCHECK(S, hipMemcpyAsync(S->d_cT, T.data(), sizeof(float) * nc, h, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_cA, A.data(), sizeof(float) * A.size(), h, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_cKab, K.data(), sizeof(float) * K.size(), h, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_inv_v0, inv.data(), sizeof(float) * inv.size(), h, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_capA, capA.data(), capA.size(), h, S->stream));
    std::vector<DrvRec> drv((size_t)S->ne * nt);
    for (int e = 0; e < S->ne; ++e)
        for (int k = 0; k < nt; ++k) {
            const size_t ck = (size_t)S->cls[e] * nt + k;
            const int h = S->col_idx[e];
            drv[(size_t)e * nt + k] = DrvRec{inv[(size_t)e * nt + k], A[ck], T[S->cls[e]], K[ck], S->len[e],
                                             S->lane_base[e],
                                             S->lanes[e] | ((S->row_ptr[h + 1] - S->row_ptr[h]) << 16),
                                             S->row_ptr[h]};
        }
    HIPCHECK(S, hipMemcpyAsync(S->d_drv, drv.data(), sizeof(DrvRec) * drv.size(), h, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_capV, capV.data(), capV.size(), h, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_cVs, VS.data(), sizeof(float) * S->ncls, hipMemcpyHostToDevice, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_cB, B.data(), sizeof(float) * S->ncls, hipMemcpyHostToDevice, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    return SIM_OK;
}

template <class T>
int h2d(sim_t* S, T* dst, const T* src, size_t n) {
    if (n == 0) return SIM_OK;
    HIPCHECK(S, hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyHostToDevice, S->stream));
    return SIM_OK;
}

int32_t tail_node(const sim_t* S, int32_t e) { return S->tail[e]; }


// With events (a sampled step), kernel q carries start event ev[2q] and stop
// event ev[2q + 1], which take that kernel's own begin and end timestamps.
#define STEP_LAUNCH_B(q, kern, grid, blk, ...)                                                            \
    do {                                                                                                 \
        if (ev)                                                                                          \
            hipExtLaunchKernelGGL(kern, grid, blk, 0, S->stream, ev[2 * (q)], ev[2 * (q) + 1], 0u, __VA_ARGS__); \
        else                                                                                             \
            hipLaunchKernelGGL(kern, grid, blk, 0, S->stream, __VA_ARGS__);                             \
    } while (0)
#define STEP_LAUNCH(q, kern, grid, ...) STEP_LAUNCH_B(q, kern, grid, b, __VA_ARGS__)

// k_decide's launch shapes: threads per block and sorted entries per thread
struct DecideShape {
    int block, per;
};
constexpr DecideShape kDecideShapes[] = {{256, 1}, {256, 2}, {128, 1}, {128, 2}, {512, 1}, {256, 4}};
constexpr int kNumDecideShapes = (int)(sizeof(kDecideShapes) / sizeof(kDecideShapes[0]));

int decide_shape_index(int block, int per) {
    for (int k = 0; k < kNumDecideShapes; ++k)
        if (kDecideShapes[k].block == block && kDecideShapes[k].per == per) return k;
    return -1;
}

int launch_step(sim_t* S, const Veh& in, const Veh& out, const Trips& tr, const Scratch& sc, const Tape& tp,
                Counters* ctr, hipEvent_t* ev) {
    const dim3 g(S->grid), gs(S->grid_small), b(kBlock);
    // kernels that read the per-XCD segments run a multiple of kSeg blocks
    const dim3 g8((S->grid + kSeg - 1) / kSeg * kSeg);
    // departure queues first, in a multiple of kSeg blocks, then the vehicles
    const int qb = tr.nq > 0 ? (S->grid_q + kSeg - 1) / kSeg * kSeg : 0;
    const dim3 gd(qb + g8.x);
    // the decide kernel with the tape, sampler and control code only when one
    // of them is on
#define DECIDE_SHAPES(F)                                                                                          \
    switch (S->dshape) {                                                                                          \
        case 1: STEP_LAUNCH_B(0, (k_decide<256, 2, F>), gd, dim3(256), S->P, S->net, tr, in, sc, tp, ctr, qb); break; \
        case 2: STEP_LAUNCH_B(0, (k_decide<128, 1, F>), gd, dim3(128), S->P, S->net, tr, in, sc, tp, ctr, qb); break; \
        case 3: STEP_LAUNCH_B(0, (k_decide<128, 2, F>), gd, dim3(128), S->P, S->net, tr, in, sc, tp, ctr, qb); break; \
        case 4: STEP_LAUNCH_B(0, (k_decide<512, 1, F>), gd, dim3(512), S->P, S->net, tr, in, sc, tp, ctr, qb); break; \
        case 5: STEP_LAUNCH_B(0, (k_decide<256, 4, F>), gd, dim3(256), S->P, S->net, tr, in, sc, tp, ctr, qb); break; \
        default: STEP_LAUNCH_B(0, (k_decide<256, 1, F>), gd, dim3(256), S->P, S->net, tr, in, sc, tp, ctr, qb); break; \
    }
    if (tp.on || sc.samp_every > 0 || S->net.ctrl)
        DECIDE_SHAPES(true)
    else
        DECIDE_SHAPES(false)
#undef DECIDE_SHAPES
    STEP_LAUNCH(1, k_resolve, g8, S->P, S->net, tr, in, sc, tp, ctr);
    STEP_LAUNCH(2, k_scan, gs, sc, ctr);
    STEP_LAUNCH(3, k_scatter, g8, S->P, in, out, sc, tp, ctr);
    STEP_LAUNCH(4, k_place, g8, S->P, tr, in, out, sc, tp, kLcNone, ctr);
    STEP_LAUNCH(5, k_lanes, g, S->P, S->net, out, sc, ctr, 1);
    HIPCHECK(S, hipGetLastError());
    return SIM_OK;
}
#undef STEP_LAUNCH

// index the lanes of a state that did not come from the previous step
int reindex(sim_t* S, const Veh& buf, const Scratch& sc, Counters* ctr) {
    hipLaunchKernelGGL(k_next_epoch, dim3(1), dim3(64), 0, S->stream, S->d_epoch);
    hipLaunchKernelGGL(k_lanes, dim3(S->grid), dim3(kBlock), 0, S->stream, S->P, S->net, buf, sc, ctr, 0);
    HIPCHECK(S, hipGetLastError());
    return SIM_OK;
}

bool alloc_veh(sim_t* S, Veh& V, size_t n) {
    return dalloc(S, V.key, n) && dalloc(S, V.x, n) && dalloc(S, V.v, n) && dalloc(S, V.edge, n) &&
           dalloc(S, V.next, n) && dalloc(S, V.lc, n) && dalloc(S, V.vid, n) && dalloc(S, V.fuel, n) &&
           dalloc(S, V.co, n) && dalloc(S, V.ty, n);
}

bool alloc_cold(sim_t* S, Cold& c, size_t n) {
    return dalloc(S, c.rcur, n) && dalloc(S, c.kin, n) && dalloc(S, c.phin, n);
}

// the step's state: the sorted vehicles (dv <- sv), their trip state by
// vehicle id (dc <- sc), departure queues, counters, stop-node holders
int copy_state(sim_t* S, const Veh& dv, const Cold& dc, int* dq, Counters* dctr, int* dhold, const Veh& sv,
               const Cold& sc, const int* sq, const Counters* sctr, const int* shold) {
    const size_t n = (size_t)S->cap;
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    HIPCHECK(S, hipMemcpyAsync(dv.key, sv.key, sizeof(int) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dv.x, sv.x, sizeof(float) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dv.v, sv.v, sizeof(float) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dv.edge, sv.edge, sizeof(int) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dv.next, sv.next, sizeof(int) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dv.lc, sv.lc, sizeof(int) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dv.vid, sv.vid, sizeof(int) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dc.rcur, sc.rcur, sizeof(int) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dc.kin, sc.kin, sizeof(int) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dc.phin, sc.phin, sizeof(float) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dv.fuel, sv.fuel, sizeof(float) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dv.co, sv.co, sizeof(float) * n, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dv.ty, sv.ty, n, k, S->stream));
    if (S->tr.nq) HIPCHECK(S, hipMemcpyAsync(dq, sq, sizeof(int) * 2 * (size_t)S->tr.nq, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dctr, sctr, sizeof(Counters), k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(dhold, shold, sizeof(int) * (size_t)S->nn, k, S->stream));
    return SIM_OK;
}

int take_checkpoint(sim_t* S, int p) {
    if (S->nckpt == S->ckpt_pool.size()) {
        sim_t::Ckpt ck;
        if (!alloc_veh(S, ck.v, S->cap) || !alloc_cold(S, ck.c, S->cap) || !dalloc(S, ck.qstate, 2 * (size_t)S->tr.nq) ||
            !dalloc(S, ck.ctr, 1) ||
            !dalloc(S, ck.holder, S->nn))
            return fail(S, SIM_ENOMEM, "checkpoint allocation failed");
        S->ckpt_pool.push_back(ck);
    }
    sim_t::Ckpt& ck = S->ckpt_pool[S->nckpt++];
    ck.t = S->host_t;
    return copy_state(S, ck.v, ck.c, ck.qstate, ck.ctr, ck.holder, S->buf[p], cold_of(S->tr), S->qstate, S->ctr,
                      S->s.holder);
}

Tape slice(sim_t* S, int k) {
    Tape t = S->slab;
    const size_t o = (size_t)k * S->cap;
    t.on = 1;
    t.x += o; t.v += o; t.vid += o; t.edge += o; t.lead += o; t.clead += o; t.next += o;
    t.mode += o; t.flags += o; t.cflags += o;
    t.n += k;
    return t;
}

void drop_graphs(sim_t* S) {
    for (auto& g : S->graphs) (void)hipGraphExecDestroy(g.exec);
    S->graphs.clear();
}

int graph_stream(sim_t* S) {
    if (S->gstream) return SIM_OK;
    HIPCHECK(S, hipStreamCreateWithFlags(&S->gstream, hipStreamNonBlocking));
    HIPCHECK(S, hipEventCreateWithFlags(&S->gjoin[0], hipEventDisableTiming));
    HIPCHECK(S, hipEventCreateWithFlags(&S->gjoin[1], hipEventDisableTiming));
    return SIM_OK;
}

template <class R>
void replay_window(sim_t* S, const ReplayCon<R>& con, int K, R* cx, R* cv, R* nx, R* nv, R* phin) {
    const dim3 g(S->adj_grid), b(kBlock);
    const sim_t::Ckpt& ck = S->ckpt_pool[0];
    hipLaunchKernelGGL(k_replay_init<R>, g, b, 0, S->stream, slice(S, 0), cx, cv, phin, (long long)S->cap);
    hipLaunchKernelGGL(k_replay_phin<R>, g, b, 0, S->stream, ck.v, ck.c.phin, ck.ctr, phin);
    hipLaunchKernelGGL(k_zero_f64, g, b, 0, S->stream, S->d_rF, (long long)S->ne);
    for (int k = 0; k < K; ++k) {
        if (k + 1 < K) hipLaunchKernelGGL(k_replay_seed<R>, g, b, 0, S->stream, slice(S, k + 1), nx, nv);
        hipLaunchKernelGGL(k_replay<R>, g, b, 0, S->stream, S->P, S->net, con, slice(S, k), cx, cv, nx, nv, phin,
                           S->d_rF, S->tr.vtype);
        std::swap(cx, nx);
        std::swap(cv, nv);
    }
}

// k_steps<R>: blocks of the whole device that run at once
template <int R>
int persistent_blocks(sim_t* S, int* out) {
    int& res = S->persist_res[R - 1];
    if (res == 0) {
        int dev = 0, cus = 0, nb = 0;
        HIPCHECK(S, hipGetDevice(&dev));
        HIPCHECK(S, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        HIPCHECK(S, hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_steps<R>, kBlock, 0));
        if (cus <= 0 || nb <= 0) return fail(S, SIM_EHIP, "the persistent step kernel cannot be resident");
        res = cus * nb;
    }
    *out = res;
    return SIM_OK;
}

// n steps in one cooperative launch of k_steps<R>
template <int R>
int launch_persistent(sim_t* S, int n) {
    int res = 0;
    int rc = persistent_blocks<R>(S, &res);
    if (rc) return rc;
    int g8 = (S->grid + kSeg - 1) / kSeg * kSeg;
    int qb = S->tr.nq > 0 ? (S->grid_q + kSeg - 1) / kSeg * kSeg : 0;
    int g = S->grid;
    const int grid = std::max(1, std::min(res, std::max(qb + g8, g)));
    int parity = (int)(S->host_t & 1);
    int lc_none = kLcNone;
    unsigned spin_limit = 1u << 20;  // about 0.05 s of polling: far above any phase
    Params P = S->P;
    Net net = S->net;
    Trips tr = S->tr;
    Veh b0 = S->buf[0], b1 = S->buf[1];
    Scratch sc = S->s;
    Counters* ctr = S->ctr;
    GridSync* gs = S->d_gsync;
    void* args[] = {&P, &net, &tr, &b0, &b1, &sc, &ctr, &gs, &n, &parity, &qb, &g8, &g, &lc_none, &spin_limit};
    // a fresh barrier count and generation (the failure flag stays until read)
    HIPCHECK(S, hipMemsetAsync(S->d_gsync, 0, 2 * sizeof(unsigned), S->stream));
    HIPCHECK(S, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_steps<R>), dim3(grid), dim3(kBlock),
                                           args, 0, S->stream));
    S->host_t += n;
    return SIM_OK;
}

int alloc_adjoint(sim_t* S) {
    if (S->adj_ready) return SIM_OK;
    const size_t cap = (size_t)S->cap, K = (size_t)S->tape_every, n = cap * K;
    Tape& t = S->slab;
    AdjState& a = S->adj;
    S->adj_grid = S->grid;
    const size_t nthreads = (size_t)S->adj_grid * kBlock;
    bool ok = alloc_veh(S, S->rbuf[0], cap) && alloc_veh(S, S->rbuf[1], cap) && alloc_cold(S, S->rcold, cap) &&
              dalloc(S, S->rqstate, 2 * (size_t)S->tr.nq) && dalloc(S, S->rctr, 1) && dalloc(S, t.x, n) && dalloc(S, t.v, n) &&
              dalloc(S, t.vid, n) && dalloc(S, t.edge, n) && dalloc(S, t.lead, n) && dalloc(S, t.clead, n) &&
              dalloc(S, t.next, n) && dalloc(S, t.mode, n) && dalloc(S, t.flags, n) && dalloc(S, t.cflags, n) &&
              dalloc(S, t.n, K) && dalloc(S, S->L0x, cap) && dalloc(S, S->L0v, cap) && dalloc(S, S->L1x, cap) &&
              dalloc(S, S->L1v, cap) && dalloc(S, a.cgx, cap) && dalloc(S, a.cgv, cap) && dalloc(S, a.cl, cap) &&
              dalloc(S, a.accx, cap) && dalloc(S, a.accv, cap) && dalloc(S, a.maxbits, 1) &&
              dalloc(S, a.scale, 1) && dalloc(S, a.lp, cap) && dalloc(S, a.gpart, nthreads * S->ncls * 4) &&
              dalloc(S, S->sink, 3 * (size_t)S->ne) && dalloc(S, S->d_rholder, S->nn) && dalloc(S, S->d_rF, S->ne);
    if (!ok) return fail(S, SIM_ENOMEM, "adjoint allocation failed");
    a.ncls = S->ncls;
    S->adj_k = S->tape_every;
    S->adj_ready = true;
    return SIM_OK;
}

// ---------------------------------------------------------------------------
// route reload (Sec. 6.3.1: each iteration simulates the horizon again with
// the re-planned routes, handed over on the device)
// ---------------------------------------------------------------------------

// the lowest trip whose route is empty, out of the table, has an edge out of
// range or two consecutive edges that do not meet
__global__ void k_route_check(const int64_t* __restrict__ ptr, const int* __restrict__ edges, long long total,
                              int ntrips, int ne, const int* __restrict__ head, const int* __restrict__ tail,
                              int* first_bad) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < ntrips; i += gridDim.x * kBlock) {
        const long long a = ptr[i], b = ptr[i + 1];
        bool ok = (i > 0 || a == 0) && 0 <= a && a < b && b <= total;
        for (long long k = a; ok && k < b; ++k) {
            const int e = edges[k];
            ok = 0 <= e && e < ne;
            if (ok && k + 1 < b) {
                const int e2 = edges[k + 1];
                ok = 0 <= e2 && e2 < ne && head[e] == tail[e2];
            }
        }
        if (!ok) atomicMin(first_bad, i);
    }
}

// per vehicle id: its route's bounds and its departure queue's key
// (first link x 4 + type), with the vehicle ids to sort by it
__global__ void k_route_trips(const int64_t* __restrict__ ptr, const int* __restrict__ edges,
                              const int* __restrict__ ord, const unsigned char* __restrict__ vtype, int n, int* rbeg,
                              int* rend, unsigned* key, int* vid) {
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const int i = ord[v];
        const long long a = ptr[i];
        rbeg[v] = (int)a;
        rend[v] = (int)ptr[i + 1];
        key[v] = 4u * (unsigned)edges[a] + vtype[v];
        vid[v] = v;
    }
}

__global__ void k_queue_flags(const unsigned* __restrict__ key, int n, int* flag) {
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < n; m += gridDim.x * kBlock)
        flag[m] = (m == 0 || key[m] != key[m - 1]) ? 1 : 0;
}

__global__ void k_queue_count(const int* __restrict__ flag, const int* __restrict__ qidx, int n, int* nq) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *nq = n > 0 ? qidx[n - 1] + flag[n - 1] : 0;
}

// the queues from the trips sorted by key (stable: by vehicle id within a
// queue): first member, link and type of each, and every member's departure
__global__ void k_queue_build(const unsigned* __restrict__ key, const int* __restrict__ qvid,
                              const int* __restrict__ flag, const int* __restrict__ qidx, const int* __restrict__ dep,
                              int n, int* qoff, int* qedge, unsigned char* qtype, int* qdep) {
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < n; m += gridDim.x * kBlock) {
        qdep[m] = dep[qvid[m]];
        if (flag[m]) {
            const int q = qidx[m];
            qoff[q] = m;
            qedge[q] = (int)(key[m] >> 2);
            qtype[q] = (unsigned char)(key[m] & 3u);
        }
        if (m == n - 1) qoff[qidx[m] + flag[m]] = n;
    }
}

__global__ void k_fill_i32(int* p, long long n, int v) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = v;
}

// the claim list's segments for nq departure queues: segment q takes the
// claims of one eighth of k_decide's tiles (at most one per vehicle; sized for
// the largest tile) and the departures of queue chunks q, q + kSeg, ...
int claim_segment(int cap, int nq) {
    const size_t vseg = ((size_t)(cap + kMaxTile - 1) / kMaxTile + kSeg - 1) / kSeg * kMaxTile;
    return (int)(vseg + ((size_t)(nq + kBlock - 1) / kBlock + kSeg - 1) / kSeg * kBlock);
}

bool alloc_claims(sim_t* S, int nq) {
    Scratch& s = S->s;
    s.cl_seg = claim_segment(S->cap, nq);
    const size_t ncl = (size_t)kSeg * s.cl_seg;
    return dalloc(S, s.cl_vid, ncl) && dalloc(S, s.cl_key, ncl) && dalloc(S, s.cl_lo, ncl) &&
           dalloc(S, s.cl_hi, ncl) && dalloc(S, s.cl_src, ncl) && dalloc(S, s.cl_kind, ncl) &&
           dalloc(S, s.cl_tedge, ncl) && dalloc(S, s.cl_cell, ncl) && dalloc(S, s.cl_X, ncl) &&
           dalloc(S, s.cl_v, ncl) && dalloc(S, s.cl_f, ncl) && dalloc(S, s.mv_claim, ncl) &&
           dalloc(S, s.mv_p, ncl) && dalloc(S, s.mv_slot, ncl) && dalloc(S, s.mv_g, ncl) &&
           dalloc(S, s.mv_src, ncl) && dalloc(S, s.mv_vid, ncl) && dalloc(S, s.mv_rc, ncl) && dalloc(S, s.mv_nx, ncl);
}

void free_claims(sim_t* S) {
    Scratch& s = S->s;
    dfree(S, s.cl_vid); dfree(S, s.cl_key); dfree(S, s.cl_lo); dfree(S, s.cl_hi); dfree(S, s.cl_src);
    dfree(S, s.cl_kind); dfree(S, s.cl_tedge); dfree(S, s.cl_cell); dfree(S, s.cl_X); dfree(S, s.cl_v);
    dfree(S, s.cl_f); dfree(S, s.mv_claim); dfree(S, s.mv_p); dfree(S, s.mv_slot); dfree(S, s.mv_g);
    dfree(S, s.mv_src); dfree(S, s.mv_vid); dfree(S, s.mv_rc); dfree(S, s.mv_nx);
}

// room for nq departure queues: the queue arrays and the claim segments
int grow_queues(sim_t* S, int nq) {
    if (nq <= S->nq_cap) return SIM_OK;
    const int cap_q = nq + nq / 4;
    dfree(S, S->tr.qoff);
    dfree(S, S->tr.qedge);
    dfree(S, S->tr.qtype);
    dfree(S, S->qstate);
    free_claims(S);
    int *qoff = nullptr, *qedge = nullptr;
    unsigned char* qtype = nullptr;
    if (!dalloc(S, qoff, (size_t)cap_q + 1) || !dalloc(S, qedge, (size_t)cap_q) || !dalloc(S, qtype, (size_t)cap_q) ||
        !dalloc(S, S->qstate, 2 * (size_t)cap_q) || !alloc_claims(S, cap_q))
        return fail(S, SIM_ENOMEM, "route reload: queue allocation failed");
    for (auto& ck : S->ckpt_pool) {  // checkpoints kept from an earlier window copy the queues too
        dfree(S, ck.qstate);
        if (!dalloc(S, ck.qstate, 2 * (size_t)cap_q)) return fail(S, SIM_ENOMEM, "route reload: queue allocation failed");
    }
    S->tr.qoff = qoff;
    S->tr.qedge = qedge;
    S->tr.qtype = qtype;
    S->nq_cap = cap_q;
    return SIM_OK;
}

}  // namespace

extern "C" {

const char* sim_strerror(int code) {
    switch (code) {
        case SIM_OK: return "ok";
        case SIM_EINVAL: return "invalid argument";
        case SIM_EROUTE: return "invalid route";
        case SIM_ENOMEM: return "out of device memory";
        case SIM_EHIP: return "HIP runtime error";
        case SIM_ESTATE: return "call not valid in the current state";
        default: return "unknown error";
    }
}

const char* sim_last_error(const sim_t* sim) { return sim ? sim->err.c_str() : "null handle"; }

int sim_create(const sim_network* net, const sim_params* prm, void* hip_stream, sim_alloc_fn alloc,
               sim_free_fn free_fn, void* alloc_ctx, sim_t** out) {
    if (!net || !prm || !out || !net->row_ptr || !net->col_idx || !net->lanes || !net->length_m ||
        !net->speed_mps || !prm->idm)
        return SIM_EINVAL;
    if ((alloc == nullptr) != (free_fn == nullptr)) return SIM_EINVAL;
    const int nn = net->num_nodes, ne = net->num_edges, ncls = prm->num_classes;
    if (nn <= 0 || ne <= 0 || ncls <= 0 || ncls > 4096 || ne >= (1 << 28)) return SIM_EINVAL;
    if (net->row_ptr[0] != 0 || net->row_ptr[nn] != ne) return SIM_EINVAL;
    for (int u = 0; u < nn; ++u)
        if (net->row_ptr[u + 1] < net->row_ptr[u]) return SIM_EINVAL;
    if (!(prm->dt > 0) || !(prm->veh_length > 0) || !(prm->s0 >= 0) || !(prm->s_eps > 0) ||
        !(prm->b_max > 0) || !(prm->mobil_bsafe >= 0) || !(prm->mand_dist >= 0) ||
        prm->lc_cooldown_steps < 0 || !std::isfinite(prm->mobil_p) || !std::isfinite(prm->mobil_athr))
        return SIM_EINVAL;

    sim_t* S = new sim_t();
    S->stream = static_cast<hipStream_t>(hip_stream);
    S->alloc = alloc;
    S->free_fn = free_fn;
    S->ctx = alloc_ctx;
    S->nn = nn;
    S->ne = ne;
    S->ncls = ncls;
    S->row_ptr.assign(net->row_ptr, net->row_ptr + nn + 1);
    S->col_idx.assign(net->col_idx, net->col_idx + ne);
    S->lanes.assign(net->lanes, net->lanes + ne);
    S->len.assign(net->length_m, net->length_m + ne);
    S->speed.assign(net->speed_mps, net->speed_mps + ne);
    S->cls.assign(ne, 0);
    if (net->link_class) S->cls.assign(net->link_class, net->link_class + ne);
    S->lane_base.resize(ne + 1);
    S->ncell.resize(ne);
    S->tail.resize(ne);
    for (int u = 0; u < nn; ++u) {
        if (S->row_ptr[u + 1] - S->row_ptr[u] > 32767) {  // packed beside the lane count in the link records
            int code = fail(S, SIM_EINVAL, "node " + std::to_string(u) + " has more than 32767 out-links");
            delete S;
            return code;
        }
        for (int e = S->row_ptr[u]; e < S->row_ptr[u + 1]; ++e) S->tail[e] = u;
    }
    std::vector<long long> cbase(ne);
    S->lane_base[0] = 0;
    long long cells = 0;
    const double min_len = (double)prm->veh_length + (double)prm->s0;
    for (int e = 0; e < ne; ++e) {
        if (S->cls[e] < 0 || S->cls[e] >= ncls || S->lanes[e] < 1 || S->lanes[e] > 8 ||
            !(S->speed[e] > 0) || !std::isfinite(S->speed[e]) || !(S->len[e] >= (float)min_len) ||
            !std::isfinite(S->len[e]) || S->col_idx[e] < 0 || S->col_idx[e] >= nn) {
            int code = fail(S, SIM_EINVAL, "edge " + std::to_string(e) + " has invalid attributes");
            delete S;
            return code;
        }
        S->ncell[e] = (int)std::floor((double)S->len[e]) + 1;
        cbase[e] = cells;
        cells += (long long)S->lanes[e] * S->ncell[e];
        S->lane_base[e + 1] = S->lane_base[e] + S->lanes[e];
    }
    S->nlanes = S->lane_base[ne];
    S->s.nlblk = (int)(((size_t)S->nlanes + (1u << kLaneBlkLog) - 1) >> kLaneBlkLog);
    S->ncells = cells;

    Params& P = S->P;
    P.dt = prm->dt;
    P.h = (float)(0.5 * (double)prm->dt * (double)prm->dt);
    P.lveh = prm->veh_length;
    P.s0 = prm->s0;
    P.claim_len = (float)((double)prm->veh_length + (double)prm->s0);
    P.s_eps = prm->s_eps;
    P.b_max = prm->b_max;
    P.pol = prm->mobil_p;
    P.athr = prm->mobil_athr;
    P.bsafe = prm->mobil_bsafe;
    P.dmand = prm->mand_dist;
    P.dt_us = std::llround((double)prm->dt * 1e6);
    P.dt_us_f = (float)((double)prm->dt * 1e6);
    P.lc_cool = prm->lc_cooldown_steps;
    P.mph = (float)(1.0 / 0.44704);
    P.nt = 1;
    P.tlen[0] = P.lveh;
    P.tclaim[0] = P.claim_len;

    float *d_len, *dummy;
    EdgeRec* d_er;
    ClaimRec* d_cr;
    int *d_lane_base, *d_lanes, *d_cls, *d_head, *d_row_ptr, *d_ncell;
    long long* d_cbase;
    // per-type constants are sized for the largest number of vehicle types (4)
    bool ok = dalloc(S, d_len, ne) && dalloc(S, S->d_inv_v0, 4 * (size_t)ne) && dalloc(S, d_lane_base, ne + 1) &&
              dalloc(S, d_lanes, ne) && dalloc(S, d_cls, ne) && dalloc(S, d_head, ne) &&
              dalloc(S, d_row_ptr, nn + 1) && dalloc(S, d_cbase, ne) && dalloc(S, d_ncell, ne) &&
              dalloc(S, S->d_capA, 4 * (size_t)ncls) && dalloc(S, S->d_capV, 4 * (size_t)ne) &&
              dalloc(S, S->d_drv, 4 * (size_t)ne) && dalloc(S, d_er, ne) && dalloc(S, d_cr, ne) &&
              dalloc(S, S->d_cT, ncls) && dalloc(S, S->d_cA, 4 * (size_t)ncls) && dalloc(S, S->d_cKab, 4 * (size_t)ncls) &&
              dalloc(S, S->d_cVs, ncls) && dalloc(S, S->d_cB, ncls) && dalloc(S, S->d_epoch, 1) &&
              dalloc(S, S->s.lanes, (size_t)S->nlanes) &&
              dalloc(S, S->s.lblk, ((size_t)S->nlanes >> kLaneBlkLog) + 2) &&
              dalloc(S, S->s.cells, (size_t)cells) && dalloc(S, S->s.st_cnt, ne) &&
              dalloc(S, S->s.st_steps, ne) && dalloc(S, S->s.st_us, ne) && dalloc(S, S->ctr, 1) &&
              dalloc(S, S->s.holder, nn) && dalloc(S, S->s.stop_req, nn) && dalloc(S, dummy, 1);
    if (!ok) {
        release_all(S);
        delete S;
        return SIM_ENOMEM;
    }
    int rc = SIM_OK;
    if ((rc = h2d(S, d_len, S->len.data(), ne)) || (rc = h2d(S, d_lane_base, S->lane_base.data(), ne + 1)) ||
        (rc = h2d(S, d_lanes, S->lanes.data(), ne)) || (rc = h2d(S, d_cls, S->cls.data(), ne)) ||
        (rc = h2d(S, d_head, S->col_idx.data(), ne)) || (rc = h2d(S, d_row_ptr, S->row_ptr.data(), nn + 1)) ||
        (rc = h2d(S, d_cbase, cbase.data(), ne)) || (rc = h2d(S, d_ncell, S->ncell.data(), ne))) {
        release_all(S);
        delete S;
        return rc;
    }
    std::vector<EdgeRec> er(ne);
    std::vector<ClaimRec> cr(ne);
    for (int e = 0; e < ne; ++e) {
        const int h = S->col_idx[e];
        er[e] = EdgeRec{S->len[e], S->lane_base[e], S->lanes[e], S->row_ptr[h]};
        cr[e] = ClaimRec{cbase[e], S->ncell[e], S->row_ptr[h + 1] - S->row_ptr[h]};
    }
    if ((rc = h2d(S, d_er, er.data(), ne)) || (rc = h2d(S, d_cr, cr.data(), ne)) ||
        (rc = (hipStreamSynchronize(S->stream) == hipSuccess ? SIM_OK : SIM_EHIP))) {
        release_all(S);
        delete S;
        return rc;
    }
    if ((rc = upload_idm(S, prm->idm)) != SIM_OK) {
        release_all(S);
        delete S;
        return rc;
    }
    hipError_t he = hipMemsetAsync(S->s.st_cnt, 0, sizeof(unsigned long long) * ne, S->stream);
    if (he == hipSuccess) he = hipMemsetAsync(S->s.st_steps, 0, sizeof(unsigned long long) * ne, S->stream);
    if (he == hipSuccess) he = hipMemsetAsync(S->s.st_us, 0, sizeof(unsigned long long) * ne, S->stream);
    if (he == hipSuccess) he = hipMemsetAsync(S->ctr, 0, sizeof(Counters), S->stream);
    if (he == hipSuccess) he = hipMemsetAsync(S->s.lanes, 0, sizeof(LaneIx) * (size_t)S->nlanes, S->stream);
    if (he == hipSuccess) {
        const unsigned one = 1u;
        he = hipMemcpyAsync(S->d_epoch, &one, sizeof(unsigned), hipMemcpyHostToDevice, S->stream);
    }
    if (he == hipSuccess) {
        int g = (int)std::min<long long>(kMaxGrid, std::max<long long>(1, (cells + kBlock - 1) / kBlock));
        hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(kBlock), 0, S->stream, S->s.cells, cells, ~0ull);
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(kBlock), 0, S->stream, S->s.stop_req, (long long)nn, ~0ull);
        he = hipGetLastError();
    }
    if (he == hipSuccess) {
        const std::vector<int> none(nn, -1);
        he = hipMemcpyAsync(S->s.holder, none.data(), sizeof(int) * nn, hipMemcpyHostToDevice, S->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(S->stream);
    }
    if (he == hipSuccess) he = hipStreamSynchronize(S->stream);
    if (he != hipSuccess) {
        release_all(S);
        delete S;
        return SIM_EHIP;
    }
    Net& N = S->net;
    N.len = d_len;
    N.inv_v0 = S->d_inv_v0;
    N.lane_base = d_lane_base;
    N.lanes = d_lanes;
    N.cls = d_cls;
    N.head = d_head;
    N.row_ptr = d_row_ptr;
    N.cbase = d_cbase;
    N.ncell = d_ncell;
    N.cT = S->d_cT;
    N.cA = S->d_cA;
    N.cKab = S->d_cKab;
    N.cVs = S->d_cVs;
    N.cB = S->d_cB;
    N.capA = S->d_capA;
    N.er = d_er;
    N.cr = d_cr;
    N.drv = S->d_drv;
    N.capV = S->d_capV;
    N.ne = ne;
    S->s.epoch = S->d_epoch;
    *out = S;
    return SIM_OK;
}

int sim_load_demand(sim_t* S, int32_t ntrips, const int32_t* depart_step, const int32_t* trip_route,
                    int32_t nroutes, const int64_t* route_ptr, const int32_t* route_edges,
                    const float* init_x, const float* init_v, const int32_t* init_lane) {
    if (!S) return SIM_EINVAL;
    if (S->loaded) return fail(S, SIM_ESTATE, "demand already loaded");
    if (ntrips < 0 || nroutes < 0 || (ntrips > 0 && (!depart_step || !trip_route || nroutes == 0)) ||
        !route_ptr || (nroutes > 0 && !route_edges))
        return fail(S, SIM_EINVAL, "null or negative demand arrays");
    if (route_ptr[0] != 0) return fail(S, SIM_EROUTE, "route_ptr[0] != 0");
    const long long nre = route_ptr[nroutes];
    if (nre < 0 || nre > (long long)INT32_MAX - 2) return fail(S, SIM_EROUTE, "route_edges too long");
    for (int r = 0; r < nroutes; ++r) {
        if (route_ptr[r + 1] <= route_ptr[r]) return fail(S, SIM_EROUTE, "empty route " + std::to_string(r));
        for (long long k = route_ptr[r]; k < route_ptr[r + 1]; ++k) {
            int e = route_edges[k];
            if (e < 0 || e >= S->ne) return fail(S, SIM_EROUTE, "edge id out of range in route " + std::to_string(r));
            if (k + 1 < route_ptr[r + 1]) {
                int e2 = route_edges[k + 1];
                if (e2 < 0 || e2 >= S->ne || S->col_idx[e] != tail_node(S, e2))
                    return fail(S, SIM_EROUTE, "route " + std::to_string(r) + " is not contiguous");
            }
        }
    }
    const int t0 = (int)S->host_t;
    int maxdep = t0;
    for (int i = 0; i < ntrips; ++i) {
        if (trip_route[i] < 0 || trip_route[i] >= nroutes) return fail(S, SIM_EINVAL, "trip_route out of range");
        if (depart_step[i] < t0) return fail(S, SIM_ESTATE, "departure before the current step");
        if (init_x && depart_step[i] != t0) return fail(S, SIM_EINVAL, "placed trips must depart now");
        maxdep = std::max(maxdep, depart_step[i]);
    }
    std::vector<int> ord(ntrips);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return depart_step[a] < depart_step[b]; });
    if (S->typed && !S->trip_type.empty() && (int)S->trip_type.size() != ntrips)
        return fail(S, SIM_EINVAL, "vehicle types were given for a different number of trips");
    std::vector<int> rbeg(ntrips), rend(ntrips), dep(ntrips);
    std::vector<unsigned char> vtype(std::max(ntrips, 1), 0);
    for (int v = 0; v < ntrips; ++v) {
        int i = ord[v];
        if (!S->trip_type.empty()) vtype[v] = S->trip_type[i];
        rbeg[v] = (int)route_ptr[trip_route[i]];
        rend[v] = (int)route_ptr[trip_route[i] + 1];
        dep[v] = depart_step[i];
    }
    const int rel_len = maxdep + 1;
    std::vector<int> rel(rel_len + 1);
    {
        int v = 0;
        for (int t = 0; t <= rel_len; ++t) {
            while (v < ntrips && dep[v] < t) ++v;
            rel[t] = v;
        }
    }
    std::vector<int> first_edge(std::max(ntrips, 1), -1);
    for (int v = 0; v < ntrips && !init_x; ++v) first_edge[v] = route_edges[rbeg[v]];
    // placed vehicles: validated, then sorted by (lane, position)
    std::vector<int> pkey, pedge, prcur, pnext, plc, pkin, pvid;
    std::vector<unsigned char> pty;
    std::vector<float> px, pv, pphin;
    if (init_x) {
        std::vector<int> idx(ntrips);
        std::vector<int> key(ntrips);
        for (int v = 0; v < ntrips; ++v) {
            int i = ord[v];
            int e = route_edges[rbeg[v]];
            int l = init_lane ? init_lane[i] : 0;
            float x = init_x[i], sp = init_v ? init_v[i] : 0.0f;
            if (l < 0 || l >= S->lanes[e] || !(x >= 0) || !(x <= S->len[e]) || !(sp >= 0) || !std::isfinite(sp))
                return fail(S, SIM_EINVAL, "placed trip " + std::to_string(i) + " out of range");
            key[v] = S->lane_base[e] + l;
            idx[v] = v;
        }
        std::sort(idx.begin(), idx.end(), [&](int a, int b) {
            if (key[a] != key[b]) return key[a] < key[b];
            float xa = init_x[ord[a]], xb = init_x[ord[b]];
            if (xa != xb) return xa < xb;
            return a < b;
        });
        for (int q = 0; q + 1 < ntrips; ++q) {
            int a = idx[q], b = idx[q + 1];
            if (key[a] == key[b] && ((init_x[ord[b]] - S->P.tlen[vtype[b]]) - init_x[ord[a]]) < 0.0f)
                return fail(S, SIM_EINVAL, "placed vehicles overlap");
        }
        for (int q = 0; q < ntrips; ++q) {
            int v = idx[q], i = ord[v];
            pkey.push_back(key[v]);
            px.push_back(init_x[i]);
            pv.push_back(init_v ? init_v[i] : 0.0f);
            pedge.push_back(route_edges[rbeg[v]]);
            prcur.push_back(rbeg[v]);
            pnext.push_back(rbeg[v] + 1 < rend[v] ? route_edges[rbeg[v] + 1] : -1);
            plc.push_back(kLcNone);
            pkin.push_back(t0);
            pphin.push_back(1.0f);
            pvid.push_back(v);
            pty.push_back(vtype[v]);
        }
    }

    // departure queues: the trips that are not placed, by (first link, type),
    // each queue by vehicle id (= by departure step)
    std::vector<int> qmem;
    qmem.reserve(ntrips);
    for (int v = 0; v < ntrips; ++v)
        if (first_edge[v] >= 0) qmem.push_back(v);
    std::stable_sort(qmem.begin(), qmem.end(), [&](int a, int b) {
        const long long ka = 4ll * first_edge[a] + vtype[a], kb = 4ll * first_edge[b] + vtype[b];
        return ka < kb;
    });
    std::vector<int> qoff(1, 0), qedge, qdep(qmem.size());
    std::vector<unsigned char> qtype;
    for (size_t m = 0; m < qmem.size(); ++m) {
        const int v = qmem[m];
        if (m == 0 || first_edge[v] != first_edge[qmem[m - 1]] || vtype[v] != vtype[qmem[m - 1]]) {
            if (m) qoff.push_back((int)m);
            qedge.push_back(first_edge[v]);
            qtype.push_back(vtype[v]);
        }
        qdep[m] = dep[v];
    }
    qoff.push_back((int)qmem.size());
    if (qmem.empty()) qoff.assign(1, 0);
    const int nq = (int)qedge.size();

    const int cap = std::max(ntrips, 1);
    S->cap = cap;
    S->ntrips = ntrips;
    int* d_re;
    int *d_rbeg, *d_rend, *d_rel;
    int *d_qoff, *d_qvid, *d_qdep, *d_qedge;
    unsigned char* d_qtype;
    Scratch& s = S->s;
    bool ok = dalloc(S, d_re, (size_t)nre) && dalloc(S, d_rbeg, cap) && dalloc(S, d_rend, cap) &&
              dalloc(S, d_rel, rel_len + 1) &&
              dalloc(S, S->tr.depart_actual, cap) && dalloc(S, S->tr.arrive_step, cap) &&
              dalloc(S, S->tr.fuel_total, cap) && dalloc(S, S->tr.co_total, cap) &&
              dalloc(S, S->d_vtype, cap) && dalloc(S, S->d_ord, cap) && dalloc(S, S->d_dep, cap) &&
              dalloc(S, d_qoff, (size_t)nq + 1) &&
              dalloc(S, d_qvid, qmem.size()) && dalloc(S, d_qdep, qmem.size()) && dalloc(S, d_qedge, (size_t)nq) &&
              dalloc(S, d_qtype, (size_t)nq) && dalloc(S, S->qstate, 2 * (size_t)nq);
    for (int b = 0; b < 2 && ok; ++b) {
        Veh& V = S->buf[b];
        ok = alloc_veh(S, V, cap);
    }
    ok = ok && dalloc(S, S->tr.rcur, cap) && dalloc(S, S->tr.kin, cap) && dalloc(S, S->tr.phin, cap);
    const size_t ntiles = (size_t)(cap + 1 + kScanTile - 1) / kScanTile + 1;
    ok = ok && dalloc(S, s.ccnt, (size_t)3 * kSeg * kSegStride) &&
         dalloc(S, s.sstat, (size_t)kSeg * kStatStride) &&
         dalloc(S, s.xs, cap) && dalloc(S, s.vs, cap) && dalloc(S, s.stay, cap + 1) &&
         dalloc(S, s.mcnt, cap + 1) && dalloc(S, s.cscan, cap + 1) && alloc_claims(S, nq) &&
         dalloc(S, s.grp_key, cap) && dalloc(S, s.grp_X, cap) && dalloc(S, s.tile_status, ntiles);
    if (!ok) return fail(S, SIM_ENOMEM, "device allocation failed in sim_load_demand");
    int rc;
    std::vector<int> minus1(cap, -1);
    if ((rc = h2d(S, d_re, route_edges, (size_t)nre)) || (rc = h2d(S, d_rbeg, rbeg.data(), ntrips)) ||
        (rc = h2d(S, d_rend, rend.data(), ntrips)) || (rc = h2d(S, d_rel, rel.data(), rel_len + 1)) ||
        (rc = h2d(S, S->d_vtype, vtype.data(), ntrips)) || (rc = h2d(S, d_qoff, qoff.data(), qoff.size())) ||
        (rc = h2d(S, d_qvid, qmem.data(), qmem.size())) || (rc = h2d(S, d_qdep, qdep.data(), qdep.size())) ||
        (rc = h2d(S, d_qedge, qedge.data(), qedge.size())) || (rc = h2d(S, d_qtype, qtype.data(), qtype.size())) ||
        (rc = h2d(S, S->tr.arrive_step, minus1.data(), cap)) || (rc = h2d(S, S->d_ord, ord.data(), ntrips)) ||
        (rc = h2d(S, S->d_dep, dep.data(), ntrips)))
        return rc;
    std::vector<int> da(cap, init_x ? t0 : -1);
    if ((rc = h2d(S, S->tr.depart_actual, da.data(), cap))) return rc;
    HIPCHECK(S, hipMemsetAsync(s.mcnt, 0, sizeof(int) * (cap + 1), S->stream));
    s.mvcnt = s.ccnt + kSeg * kSegStride;
    s.tcnt = s.ccnt + 2 * kSeg * kSegStride;
    HIPCHECK(S, hipMemsetAsync(s.ccnt, 0, sizeof(int) * 3 * kSeg * kSegStride, S->stream));
    HIPCHECK(S, hipMemsetAsync(s.sstat, 0, sizeof(unsigned long long) * kSeg * kStatStride, S->stream));
    if (nq) HIPCHECK(S, hipMemsetAsync(S->qstate, 0, sizeof(int) * 2 * (size_t)nq, S->stream));
    HIPCHECK(S, hipMemsetAsync(S->tr.fuel_total, 0, sizeof(float) * cap, S->stream));
    HIPCHECK(S, hipMemsetAsync(S->tr.co_total, 0, sizeof(float) * cap, S->stream));
    for (int b = 0; b < 2; ++b) {
        HIPCHECK(S, hipMemsetAsync(S->buf[b].fuel, 0, sizeof(float) * cap, S->stream));
        HIPCHECK(S, hipMemsetAsync(S->buf[b].co, 0, sizeof(float) * cap, S->stream));
    }
    HIPCHECK(S, hipMemsetAsync(s.stay, 0, cap + 1, S->stream));
    HIPCHECK(S, hipMemsetAsync(s.tile_status, 0, sizeof(unsigned long long) * ntiles, S->stream));
    const int p = (int)(S->host_t & 1);
    const int np = (int)pkey.size();
    {  // trip state by vehicle id: the placed vehicles', the rest set at departure
        std::vector<int> crcur(cap, 0), ckin(cap, 0);
        std::vector<float> cphin(cap, 1.0f);
        for (int i = 0; i < np; ++i) {
            crcur[pvid[i]] = prcur[i];
            ckin[pvid[i]] = pkin[i];
            cphin[pvid[i]] = pphin[i];
        }
        if ((rc = h2d(S, S->tr.rcur, crcur.data(), cap)) || (rc = h2d(S, S->tr.kin, ckin.data(), cap)) ||
            (rc = h2d(S, S->tr.phin, cphin.data(), cap)))
            return rc;
    }
    if (np) {
        Veh& V = S->buf[p];
        if ((rc = h2d(S, V.key, pkey.data(), np)) || (rc = h2d(S, V.x, px.data(), np)) ||
            (rc = h2d(S, V.v, pv.data(), np)) || (rc = h2d(S, V.edge, pedge.data(), np)) ||
            (rc = h2d(S, V.next, pnext.data(), np)) || (rc = h2d(S, V.lc, plc.data(), np)) ||
            (rc = h2d(S, V.vid, pvid.data(), np)) || (rc = h2d(S, V.ty, pty.data(), np)))
            return rc;
    }
    Counters c0{};
    c0.t = t0;
    c0.n = np;
    c0.departed = (unsigned long long)np;
    HIPCHECK(S, hipMemcpyAsync(S->ctr, &c0, sizeof(Counters), hipMemcpyHostToDevice, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    S->tr.route_edges = d_re;
    S->tr.rbeg = d_rbeg;
    S->tr.rend = d_rend;
    S->tr.rel_off = d_rel;
    S->tr.rel_len = rel_len;
    S->tr.vtype = S->d_vtype;
    S->tr.nq = nq;
    S->tr.qoff = d_qoff;
    S->tr.qvid = d_qvid;
    S->tr.qdep = d_qdep;
    S->tr.qedge = d_qedge;
    S->tr.qtype = d_qtype;
    S->tr.qhead = S->qstate;
    S->tr.qtail = S->qstate + nq;
    S->h_rbeg = rbeg;
    S->t_load = t0;
    S->placed = init_x != nullptr;
    S->re_cap = nre;
    S->nq_cap = nq;
    S->grid = (int)std::min<long long>(kMaxGrid, std::max<long long>(1, ((long long)cap + kBlock - 1) / kBlock));
    S->grid_small = std::max(1, S->grid / 4);
    S->grid_q = (int)std::min<long long>(kMaxGrid, std::max<long long>(1, ((long long)nq + kBlock - 1) / kBlock));
    if ((rc = reindex(S, S->buf[p], S->s, S->ctr))) return rc;
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    S->loaded = true;
    return SIM_OK;
}

int sim_step(sim_t* S, int32_t num_steps) {
    if (!S) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    if (num_steps < 0) return fail(S, SIM_EINVAL, "negative step count");
    const Tape off{};
    for (int k = 0; k < num_steps; ++k) {
        const int p = (int)(S->host_t & 1);
        if (S->tape_on && (S->host_t - S->tape_t0) % S->tape_every == 0) {
            int rc = take_checkpoint(S, p);
            if (rc) return rc;
        }
        hipEvent_t ev[2 * SIM_NUM_KERNELS] = {};
        const bool timed = S->timing_every > 0 && (S->host_t % S->timing_every) == 0;
        if (timed) {
            for (int q = 0; q < 2 * SIM_NUM_KERNELS; ++q) {
                if (S->ev_free.empty()) {
                    hipEvent_t e;
                    HIPCHECK(S, hipEventCreate(&e));
                    S->ev_free.push_back(e);
                }
                ev[q] = S->ev_free.back();
                S->ev_free.pop_back();
            }
        }
        int rc = launch_step(S, S->buf[p], S->buf[p ^ 1], S->tr, S->s, off, S->ctr,
                             timed ? ev : nullptr);
        if (rc) return rc;
        if (timed) S->ev_steps.emplace_back(ev, ev + 2 * SIM_NUM_KERNELS);
        S->host_t += 1;
    }
    return SIM_OK;
}

int sim_step_persistent(sim_t* S, int32_t num_steps) {
    if (!S) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    if (num_steps < 0) return fail(S, SIM_EINVAL, "negative step count");
    if (S->tape_on || S->timing_every > 0) return sim_step(S, num_steps);  // per-step host work: plain launches
    if (kDecideShapes[S->dshape].block != kBlock || kDecideShapes[S->dshape].per > 2)
        return fail(S, SIM_EINVAL, "the persistent step takes decide shapes of 256 threads and 1 or 2 entries each");
    if (!S->d_gsync) {
        if (!dalloc(S, S->d_gsync, 1)) return fail(S, SIM_ENOMEM, "barrier state");
        HIPCHECK(S, hipMemsetAsync(S->d_gsync, 0, sizeof(GridSync), S->stream));
    }
    // at most 600 steps per launch
    for (int done = 0; done < num_steps;) {
        const int n = std::min(600, num_steps - done);
        const int rc = kDecideShapes[S->dshape].per == 2 ? launch_persistent<2>(S, n) : launch_persistent<1>(S, n);
        if (rc) return rc;
        done += n;
    }
    GridSync h{};
    HIPCHECK(S, hipMemcpyAsync(&h, S->d_gsync, sizeof(GridSync), hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    if (h.fail) return fail(S, SIM_EHIP, "a device-wide barrier of the persistent step gave up waiting: state void");
    return SIM_OK;
}

int sim_tape_begin(sim_t* S, int32_t checkpoint_every) {
    if (!S || checkpoint_every <= 0) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    if (S->ncls > 16) return fail(S, SIM_EINVAL, "differentiation supports at most 16 link classes");
    if (S->adj_ready && checkpoint_every > S->adj_k)
        return fail(S, SIM_EINVAL, "checkpoint interval larger than the one the adjoint buffers were sized for");
    S->tape_on = true;
    S->tape_full_t = -1;
    S->tape_t0 = S->host_t;
    S->tape_every = checkpoint_every;
    S->nckpt = 0;
    return SIM_OK;
}

// The recompute pass of a differentiation window: statistics into a sink, no
// samples, stop-node admissions and departure queues on their own copies, so
// the live state is untouched.
Scratch recompute_scratch(sim_t* S) {
    Scratch rs = S->s;
    rs.samp_every = 0;
    rs.st_cnt = S->sink;
    rs.st_steps = S->sink + S->ne;
    rs.st_us = S->sink + 2 * (size_t)S->ne;
    rs.holder = S->d_rholder;
    return rs;
}

Trips recompute_trips(sim_t* S) {
    Trips rtr = S->tr;
    rtr.qhead = S->rqstate;
    rtr.qtail = S->rqstate + S->tr.nq;
    rtr.rcur = S->rcold.rcur;
    rtr.kin = S->rcold.kin;
    rtr.phin = S->rcold.phin;
    return rtr;
}

// segment c of the window recomputed from its checkpoint with the event tape on
int recompute_segment(sim_t* S, size_t c, const Scratch& rs, const Trips& rtr, int* K_out) {
    const sim_t::Ckpt& ck = S->ckpt_pool[c];
    const long long t_end = (c + 1 < S->nckpt) ? S->ckpt_pool[c + 1].t : S->host_t;
    const int K = (int)(t_end - ck.t);
    int rc;
    if ((rc = copy_state(S, S->rbuf[0], S->rcold, S->rqstate, S->rctr, S->d_rholder, ck.v, ck.c, ck.qstate, ck.ctr,
                         ck.holder)))
        return rc;
    if ((rc = reindex(S, S->rbuf[0], rs, S->rctr))) return rc;
    for (int k = 0; k < K; ++k)
        if ((rc = launch_step(S, S->rbuf[k & 1], S->rbuf[(k + 1) & 1], rtr, rs, slice(S, k), S->rctr, nullptr)))
            return rc;
    *K_out = K;
    return SIM_OK;
}

// a window of one segment: its whole tape into the slices
int record_window(sim_t* S) {
    int K = 0;
    int rc = recompute_segment(S, 0, recompute_scratch(S), recompute_trips(S), &K);
    if (rc) return rc;
    S->tape_full_t = S->host_t;
    // the recompute pass re-indexed the lanes: index the live state again
    return reindex(S, S->buf[S->host_t & 1], S->s, S->ctr);
}

int sim_grad(sim_t* S, const float* dL_dmeanTT, float* dL_dtheta) {
    if (!S || !dL_dmeanTT || !dL_dtheta) return SIM_EINVAL;
    if (!S->tape_on) return fail(S, SIM_ESTATE, "sim_grad without sim_tape_begin");
    int rc = alloc_adjoint(S);
    if (rc) return rc;
    const int G = S->adj_grid;
    const int nvals = S->ncls * 4;
    const long long nthreads = (long long)G * kBlock;
    const dim3 g(G), b(kBlock);
    hipLaunchKernelGGL(k_zero_f64, g, b, 0, S->stream, S->adj.gpart, nthreads * nvals);
    hipLaunchKernelGGL(k_zero_f32, g, b, 0, S->stream, S->adj.lp, (long long)S->cap);
    hipLaunchKernelGGL(k_zero_f32, g, b, 0, S->stream, S->L1x, (long long)S->cap);
    hipLaunchKernelGGL(k_zero_f32, g, b, 0, S->stream, S->L1v, (long long)S->cap);
    hipLaunchKernelGGL(k_zero_i64, g, b, 0, S->stream, S->adj.accx, (long long)S->cap);
    hipLaunchKernelGGL(k_zero_i64, g, b, 0, S->stream, S->adj.accv, (long long)S->cap);
    HIPCHECK(S, hipMemsetAsync(S->adj.maxbits, 0, sizeof(unsigned), S->stream));
    HIPCHECK(S, hipGetLastError());
    const Scratch rs = recompute_scratch(S);
    const Trips rtr = recompute_trips(S);
    AdjState a = S->adj;
    a.vtype = S->tr.vtype;
    a.dLdT = dL_dmeanTT;
    a.cnt = S->s.st_cnt;
    float *L0x = S->L0x, *L0v = S->L0v, *L1x = S->L1x, *L1v = S->L1v;
    for (size_t c = S->nckpt; c-- > 0;) {
        int K = 0;
        if ((rc = recompute_segment(S, c, rs, rtr, &K))) return rc;
        for (int k = K - 1; k >= 0; --k) {
            const Tape tk = slice(S, k);
            a.L1x = L1x;
            a.L1v = L1v;
            a.L0x = L0x;
            a.L0v = L0v;
            hipLaunchKernelGGL(k_adj_own, g, b, 0, S->stream, S->P, S->net, tk, a);
            hipLaunchKernelGGL(k_adj_lead, g, b, 0, S->stream, tk, a);
            hipLaunchKernelGGL(k_adj_sum, g, b, 0, S->stream, tk, a);
            HIPCHECK(S, hipGetLastError());
            std::swap(L0x, L1x);
            std::swap(L0v, L1v);
        }
    }
    // one segment: its tape, now in the slices, covers the whole window
    S->tape_full_t = S->nckpt == 1 ? S->host_t : -1;
    // the recompute pass re-indexed the lanes: index the live state again
    if ((rc = reindex(S, S->buf[S->host_t & 1], S->s, S->ctr))) return rc;
    double* out64 = nullptr;
    hipLaunchKernelGGL(k_adj_reduce, dim3((nvals + 63) / 64), dim3(64), 0, S->stream, S->adj.gpart, (int)nthreads,
                       nvals, dL_dtheta, out64);
    HIPCHECK(S, hipGetLastError());
    return SIM_OK;
}

int sim_replay(sim_t* S, const double* idm, int32_t fp64, double* frac_sum) {
    if (!S || !idm || !frac_sum) return SIM_EINVAL;
    if (!S->tape_on || S->nckpt != 1)
        return fail(S, SIM_ESTATE, "sim_replay needs a window recorded as one segment (sim_tape_begin with a "
                                   "checkpoint interval at least its length)");
    const int nt = S->P.nt, nc = S->ncls;
    for (int c = 0; c < nc; ++c) {
        const double s0 = idm[4 * c + 0], t = idm[4 * c + 1], a = idm[4 * c + 2], b = idm[4 * c + 3];
        if (!(s0 > 0) || !(t >= 0) || !(a > 0) || !(b > 0) || !std::isfinite(s0 * t * a * b))
            return fail(S, SIM_EINVAL, "idm parameters of class " + std::to_string(c) + " out of range");
    }
    int rc = alloc_adjoint(S);
    if (rc) return rc;
    const int K = (int)(S->host_t - S->ckpt_pool[0].t);
    if (K > S->adj_k) return fail(S, SIM_ESTATE, "window longer than the tape buffers");
    if (S->tape_full_t != S->host_t && (rc = record_window(S))) return rc;
    if (fp64) {
        // the constants in double from the parameters, in the expressions the
        // float ones are rounded from
        const size_t ncon = (size_t)nc * nt * 2 + nc + (size_t)S->ne * nt;
        if (!S->d_r64 && !(dalloc(S, S->d_r64, 5 * (size_t)S->cap) && dalloc(S, S->d_r64c, ncon)))
            return fail(S, SIM_ENOMEM, "replay buffers");
        std::vector<double> con(ncon);
        double *A = con.data(), *Kb = A + (size_t)nc * nt, *T = Kb + (size_t)nc * nt, *iv = T + nc;
        for (int c = 0; c < nc; ++c) {
            const double a = idm[4 * c + 2], b = idm[4 * c + 3];
            T[c] = idm[4 * c + 1];
            for (int k = 0; k < nt; ++k) {
                const double ak = a < S->tamax[k] ? a : S->tamax[k];
                A[(size_t)c * nt + k] = ak;
                Kb[(size_t)c * nt + k] = 1.0 / (2.0 * std::sqrt(ak * b));
            }
        }
        for (int e = 0; e < S->ne; ++e) {
            const double v0 = idm[4 * S->cls[e] + 0] * (double)S->speed[e];
            for (int k = 0; k < nt; ++k) iv[(size_t)e * nt + k] = 1.0 / (v0 < S->tvmax[k] ? v0 : S->tvmax[k]);
        }
        HIPCHECK(S, hipMemcpyAsync(S->d_r64c, con.data(), sizeof(double) * ncon, hipMemcpyHostToDevice, S->stream));
        double* dc = S->d_r64c;
        const ReplayCon<double> rc64{dc, dc + 2 * (size_t)nc * nt, dc + (size_t)nc * nt, dc + 2 * (size_t)nc * nt + nc};
        double* r = S->d_r64;
        const size_t c = (size_t)S->cap;
        replay_window<double>(S, rc64, K, r, r + c, r + 2 * c, r + 3 * c, r + 4 * c);
        HIPCHECK(S, hipGetLastError());
        HIPCHECK(S, hipMemcpyAsync(frac_sum, S->d_rF, sizeof(double) * S->ne, hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipStreamSynchronize(S->stream));  // also keeps the host constants alive for their copy
        return SIM_OK;
    }
    // in float: the simulator's own constants at these parameters, then the
    // live ones back
    const std::vector<float> keep = S->idm_in;
    std::vector<float> f32(idm, idm + 4 * (size_t)nc);
    if ((rc = upload_idm(S, f32.data()))) return rc;
    const ReplayCon<float> rc32{S->net.cA, S->net.cT, S->net.cKab, S->net.inv_v0};
    replay_window<float>(S, rc32, K, S->L0x, S->L0v, S->L1x, S->L1v, S->adj.lp);
    hipError_t he = hipGetLastError();
    if (he == hipSuccess)
        he = hipMemcpyAsync(frac_sum, S->d_rF, sizeof(double) * S->ne, hipMemcpyDeviceToHost, S->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(S->stream);
    const int rc2 = upload_idm(S, keep.data());
    if (he != hipSuccess) {
        (void)hipGetLastError();
        return fail(S, SIM_EHIP, std::string("sim_replay: ") + hipGetErrorString(he));
    }
    return rc2;
}

int sim_stats(sim_t* S, sim_stats_t* host_out, int64_t* edge_count, int64_t* edge_tt_steps, int64_t* edge_tt_us) {
    if (!S) return SIM_EINVAL;
    if (edge_count)
        HIPCHECK(S, hipMemcpyAsync(edge_count, S->s.st_cnt, sizeof(int64_t) * S->ne, hipMemcpyDeviceToDevice, S->stream));
    if (edge_tt_steps)
        HIPCHECK(S, hipMemcpyAsync(edge_tt_steps, S->s.st_steps, sizeof(int64_t) * S->ne, hipMemcpyDeviceToDevice, S->stream));
    if (edge_tt_us)
        HIPCHECK(S, hipMemcpyAsync(edge_tt_us, S->s.st_us, sizeof(int64_t) * S->ne, hipMemcpyDeviceToDevice, S->stream));
    if (host_out) {
        Counters c{};
        if (S->ctr) {
            HIPCHECK(S, hipMemcpyAsync(&c, S->ctr, sizeof(Counters), hipMemcpyDeviceToHost, S->stream));
            HIPCHECK(S, hipStreamSynchronize(S->stream));
        }
        host_out->step = S->loaded ? c.t : S->host_t;
        host_out->loaded = S->ntrips;
        host_out->en_route = c.n;
        host_out->arrived = (int64_t)c.arrived;
        host_out->departed = (int64_t)c.departed;
        host_out->waiting = (int64_t)S->ntrips - (int64_t)c.departed;
        host_out->vehicle_updates = (int64_t)c.updates;
        host_out->claims_lost = (int64_t)c.claims_lost;
        host_out->clamps = (int64_t)c.clamps;
        host_out->claims = (int64_t)c.claims;
        host_out->claims_departure = (int64_t)c.claims_dep;
        host_out->lc_evaluated = (int64_t)c.lc_eval;
        host_out->claims_lane_change = (int64_t)c.claims_lc;
    }
    return SIM_OK;
}

int sim_read_vehicles(sim_t* S, int32_t cap, int32_t* n_out, int32_t* vid, int32_t* edge, int32_t* lane,
                      int32_t* cursor, int32_t* lc, int32_t* kin, float* x, float* v, float* phin, float* fuel,
                      float* co) {
    if (!S || !n_out || cap < 0) return SIM_EINVAL;
    if (!S->loaded) {
        *n_out = 0;
        return SIM_OK;
    }
    Counters c{};
    HIPCHECK(S, hipMemcpyAsync(&c, S->ctr, sizeof(Counters), hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    *n_out = c.n;
    if (c.n > cap) return fail(S, SIM_EINVAL, "capacity too small");
    const int n = c.n;
    const Veh& V = S->buf[S->host_t & 1];
    std::vector<int> hvid(n), hedge(n), hkey(n);
    // the trip state is kept by vehicle id: whole arrays, read only if asked for
    std::vector<int> crcur(cursor ? S->cap : 0), ckin(kin ? S->cap : 0);
    std::vector<float> cphin(phin ? S->cap : 0);
    if (n) {
        HIPCHECK(S, hipMemcpyAsync(hvid.data(), V.vid, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipMemcpyAsync(hedge.data(), V.edge, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipMemcpyAsync(hkey.data(), V.key, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        const size_t cb = sizeof(int) * (size_t)S->cap;
        if (cursor) HIPCHECK(S, hipMemcpyAsync(crcur.data(), S->tr.rcur, cb, hipMemcpyDeviceToHost, S->stream));
        if (kin) HIPCHECK(S, hipMemcpyAsync(ckin.data(), S->tr.kin, cb, hipMemcpyDeviceToHost, S->stream));
        if (phin) HIPCHECK(S, hipMemcpyAsync(cphin.data(), S->tr.phin, cb, hipMemcpyDeviceToHost, S->stream));
        if (lc) HIPCHECK(S, hipMemcpyAsync(lc, V.lc, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        if (x) HIPCHECK(S, hipMemcpyAsync(x, V.x, sizeof(float) * n, hipMemcpyDeviceToHost, S->stream));
        if (v) HIPCHECK(S, hipMemcpyAsync(v, V.v, sizeof(float) * n, hipMemcpyDeviceToHost, S->stream));
        if (fuel) HIPCHECK(S, hipMemcpyAsync(fuel, V.fuel, sizeof(float) * n, hipMemcpyDeviceToHost, S->stream));
        if (co) HIPCHECK(S, hipMemcpyAsync(co, V.co, sizeof(float) * n, hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipStreamSynchronize(S->stream));
    }
    for (int i = 0; i < n; ++i) {
        const int id = hvid[i];
        if (vid) vid[i] = id;
        if (edge) edge[i] = hedge[i];
        if (lane) lane[i] = hkey[i] - S->lane_base[hedge[i]];
        if (cursor) cursor[i] = crcur[id] - S->h_rbeg[id];
        if (kin) kin[i] = ckin[id];
        if (phin) phin[i] = cphin[id];
    }
    return SIM_OK;
}

int sim_read_trips(sim_t* S, int32_t* depart_actual, int32_t* arrive_step) {
    if (!S) return SIM_EINVAL;
    if (!S->loaded || S->ntrips == 0) return SIM_OK;
    if (depart_actual)
        HIPCHECK(S, hipMemcpyAsync(depart_actual, S->tr.depart_actual, sizeof(int) * S->ntrips, hipMemcpyDeviceToHost, S->stream));
    if (arrive_step)
        HIPCHECK(S, hipMemcpyAsync(arrive_step, S->tr.arrive_step, sizeof(int) * S->ntrips, hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    return SIM_OK;
}

// ---------------------------------------------------------------------------
// state image: a header, then the sections below, each 256-byte aligned
// ---------------------------------------------------------------------------
namespace {
constexpr unsigned long long kStateMagic = 0x3254415453534D54ull;  // "TMSSTAT2"
struct StateHdr {
    unsigned long long magic;
    long long step, cap, nq, nn, ne, ntrips, bytes;
};
struct StateLayout {
    size_t veh[13];
    size_t q, ctr, hold, trip[4], st[3], total;
};
StateLayout state_layout(const sim_t* S) {
    StateLayout L{};
    size_t o = 256;  // the header
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 255) / 256 * 256;
        return at;
    };
    const size_t n = (size_t)S->cap;
    for (int f = 0; f < 12; ++f) L.veh[f] = take(4 * n);
    L.veh[12] = take(n);
    L.q = take(sizeof(int) * 2 * (size_t)S->tr.nq);
    L.ctr = take(sizeof(Counters));
    L.hold = take(sizeof(int) * (size_t)S->nn);
    for (int f = 0; f < 4; ++f) L.trip[f] = take(4 * n);
    for (int f = 0; f < 3; ++f) L.st[f] = take(sizeof(unsigned long long) * (size_t)S->ne);
    L.total = o;
    return L;
}
// the 13 vehicle arrays, in image order: the sorted arrays of a buffer and
// (route cursor, entry step, entry fraction) the trip state by vehicle id
void veh_fields(const Veh& V, const Trips& T, void* f[13]) {
    void* a[13] = {V.key, V.x, V.v, V.edge, T.rcur, V.next, V.lc, T.kin, T.phin, V.vid, V.fuel, V.co, V.ty};
    for (int i = 0; i < 13; ++i) f[i] = a[i];
}

const char* const kCheckNames[kChkClasses] = {
    "vehicle count or step", "lane key", "link of the lane key", "order by (lane, position)", "position", "speed",
    "vehicle id", "duplicate vehicle id", "vehicle type", "route cursor", "next link", "entry fraction, fuel or CO",
    "arrived vehicle on the road", "departure queue", "stop-node holder"};
static_assert(kChkClasses == SIM_CHECK_CLASSES, "the check classes are the public ones");

// One pass of k_check_state over a state (c.n vehicles at step t); counts and
// first receive, per class, the violations and the lowest offending entry.
// A count or step out of range is reported without reading any array.
int check_state(sim_t* S, const CheckIn& c, int t, unsigned long long* counts, int* first) {
    for (int k = 0; k < kChkClasses; ++k) {
        counts[k] = 0;
        first[k] = INT32_MAX;
    }
    if (c.n < 0 || c.n > S->cap || t < 0) {
        counts[kChkCount] = 1;
        first[kChkCount] = 0;
        return SIM_OK;
    }
    const size_t words = ((size_t)S->cap + 31) / 32;
    if (!S->d_chk_seen && !(dalloc(S, S->d_chk_seen, words) && dalloc(S, S->d_chk_fail, (size_t)kChkClasses) &&
                            dalloc(S, S->d_chk_first, (size_t)kChkClasses)))
        return fail(S, SIM_ENOMEM, "state check: device allocation failed");
    HIPCHECK(S, hipMemsetAsync(S->d_chk_seen, 0, sizeof(unsigned) * words, S->stream));
    HIPCHECK(S, hipMemsetAsync(S->d_chk_fail, 0, sizeof(unsigned long long) * kChkClasses, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_chk_first, first, sizeof(int) * kChkClasses, hipMemcpyHostToDevice, S->stream));
    const long long items = std::max<long long>({(long long)c.n, (long long)S->tr.nq, (long long)S->nn, 1ll});
    const dim3 g((unsigned)std::min<long long>(kMaxGrid, (items + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_check_state, g, dim3(kBlock), 0, S->stream, c, S->net, S->tr, S->nlanes, S->P.nt,
                       S->ntrips, S->nn, S->d_chk_seen, S->d_chk_fail, S->d_chk_first);
    HIPCHECK(S, hipGetLastError());
    HIPCHECK(S, hipMemcpyAsync(counts, S->d_chk_fail, sizeof(unsigned long long) * kChkClasses,
                               hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipMemcpyAsync(first, S->d_chk_first, sizeof(int) * kChkClasses, hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    return SIM_OK;
}
}  // namespace

int sim_state_bytes(sim_t* S, size_t* bytes) {
    if (!S || !bytes) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    *bytes = state_layout(S).total;
    return SIM_OK;
}

int sim_get_state(sim_t* S, sim_state_view* out, void* image) {
    if (!S || !out) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    const Veh& V = S->buf[S->host_t & 1];
    if (image) {
        const StateLayout L = state_layout(S);
        char* img = static_cast<char*>(image);
        const hipMemcpyKind k = hipMemcpyDeviceToDevice;
        const size_t n = (size_t)S->cap;
        void* f[13];
        veh_fields(V, S->tr, f);
        for (int i = 0; i < 13; ++i) HIPCHECK(S, hipMemcpyAsync(img + L.veh[i], f[i], i < 12 ? 4 * n : n, k, S->stream));
        if (S->tr.nq) HIPCHECK(S, hipMemcpyAsync(img + L.q, S->qstate, sizeof(int) * 2 * (size_t)S->tr.nq, k, S->stream));
        HIPCHECK(S, hipMemcpyAsync(img + L.ctr, S->ctr, sizeof(Counters), k, S->stream));
        HIPCHECK(S, hipMemcpyAsync(img + L.hold, S->s.holder, sizeof(int) * (size_t)S->nn, k, S->stream));
        const void* tf[4] = {S->tr.depart_actual, S->tr.arrive_step, S->tr.fuel_total, S->tr.co_total};
        for (int i = 0; i < 4; ++i) HIPCHECK(S, hipMemcpyAsync(img + L.trip[i], tf[i], 4 * n, k, S->stream));
        const void* sf[3] = {S->s.st_cnt, S->s.st_steps, S->s.st_us};
        for (int i = 0; i < 3; ++i)
            HIPCHECK(S, hipMemcpyAsync(img + L.st[i], sf[i], sizeof(unsigned long long) * (size_t)S->ne, k, S->stream));
        const StateHdr h{kStateMagic, S->host_t, S->cap, S->tr.nq, S->nn, S->ne, S->ntrips, (long long)L.total};
        HIPCHECK(S, hipMemcpyAsync(img, &h, sizeof(h), hipMemcpyHostToDevice, S->stream));
        HIPCHECK(S, hipStreamSynchronize(S->stream));  // before h goes out of scope
    }
    Counters c{};
    HIPCHECK(S, hipMemcpyAsync(&c, S->ctr, sizeof(Counters), hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    out->step = S->host_t;
    out->num_vehicles = c.n;
    out->key = V.key;
    out->x = V.x;
    out->v = V.v;
    out->edge = V.edge;
    out->vid = V.vid;
    out->type = V.ty;
    return SIM_OK;
}

int sim_set_state(sim_t* S, const void* image, size_t bytes) {
    if (!S || !image) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    if (S->tape_on || S->adj_ready) return fail(S, SIM_ESTATE, "no state replacement inside a differentiation window");
    const StateLayout L = state_layout(S);
    if (bytes != L.total) return fail(S, SIM_EINVAL, "state image size does not match this simulation");
    StateHdr h{};
    HIPCHECK(S, hipMemcpyAsync(&h, image, sizeof(h), hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    if (h.magic != kStateMagic || h.cap != S->cap || h.nq != S->tr.nq || h.nn != S->nn || h.ne != S->ne ||
        h.ntrips != S->ntrips || h.bytes != (long long)L.total || h.step < 0)
        return fail(S, SIM_EINVAL, "not a state image of this simulation");
    const char* img = static_cast<const char*>(image);
    {  // the image's contents, checked in place before any of it is copied in
        Counters hc{};
        HIPCHECK(S, hipMemcpyAsync(&hc, img + L.ctr, sizeof(Counters), hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipStreamSynchronize(S->stream));
        auto at = [&](int f) { return img + L.veh[f]; };
        CheckIn c;
        c.key = reinterpret_cast<const int*>(at(0));
        c.x = reinterpret_cast<const float*>(at(1));
        c.v = reinterpret_cast<const float*>(at(2));
        c.edge = reinterpret_cast<const int*>(at(3));
        c.rcur = reinterpret_cast<const int*>(at(4));
        c.next = reinterpret_cast<const int*>(at(5));
        c.phin = reinterpret_cast<const float*>(at(8));
        c.vid = reinterpret_cast<const int*>(at(9));
        c.fuel = reinterpret_cast<const float*>(at(10));
        c.co = reinterpret_cast<const float*>(at(11));
        c.ty = reinterpret_cast<const unsigned char*>(at(12));
        c.arrive = reinterpret_cast<const int*>(img + L.trip[1]);
        c.qstate = reinterpret_cast<const int*>(img + L.q);
        c.holder = reinterpret_cast<const int*>(img + L.hold);
        c.n = hc.n;
        unsigned long long cnt[kChkClasses];
        int first[kChkClasses];
        const int rc = check_state(S, c, hc.t, cnt, first);
        if (rc) return rc;
        for (int k = 0; k < kChkClasses; ++k)
            if (cnt[k])
                return fail(S, SIM_EINVAL, std::string("state image fails validation: ") + kCheckNames[k] + " (" +
                                               std::to_string(cnt[k]) + " cases, first at " +
                                               std::to_string(first[k]) + ")");
    }
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    const size_t n = (size_t)S->cap;
    const int p = (int)(h.step & 1);
    void* f[13];
    veh_fields(S->buf[p], S->tr, f);
    for (int i = 0; i < 13; ++i) HIPCHECK(S, hipMemcpyAsync(f[i], img + L.veh[i], i < 12 ? 4 * n : n, k, S->stream));
    if (S->tr.nq) HIPCHECK(S, hipMemcpyAsync(S->qstate, img + L.q, sizeof(int) * 2 * (size_t)S->tr.nq, k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->ctr, img + L.ctr, sizeof(Counters), k, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->s.holder, img + L.hold, sizeof(int) * (size_t)S->nn, k, S->stream));
    void* tf[4] = {S->tr.depart_actual, S->tr.arrive_step, S->tr.fuel_total, S->tr.co_total};
    for (int i = 0; i < 4; ++i) HIPCHECK(S, hipMemcpyAsync(tf[i], img + L.trip[i], 4 * n, k, S->stream));
    void* sf[3] = {S->s.st_cnt, S->s.st_steps, S->s.st_us};
    for (int i = 0; i < 3; ++i)
        HIPCHECK(S, hipMemcpyAsync(sf[i], img + L.st[i], sizeof(unsigned long long) * (size_t)S->ne, k, S->stream));
    S->host_t = h.step;
    int rc = reindex(S, S->buf[p], S->s, S->ctr);
    if (rc) return rc;
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    return SIM_OK;
}

int sim_check_state(sim_t* S, int64_t* counts, int32_t* first) {
    if (!S || !counts) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    const Veh& V = S->buf[S->host_t & 1];
    Counters hc{};
    HIPCHECK(S, hipMemcpyAsync(&hc, S->ctr, sizeof(Counters), hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    CheckIn c;
    c.key = V.key;
    c.x = V.x;
    c.v = V.v;
    c.edge = V.edge;
    c.next = V.next;
    c.vid = V.vid;
    c.fuel = V.fuel;
    c.co = V.co;
    c.ty = V.ty;
    c.rcur = S->tr.rcur;
    c.phin = S->tr.phin;
    c.arrive = S->tr.arrive_step;
    c.qstate = S->qstate;
    c.holder = S->s.holder;
    c.n = hc.n;
    unsigned long long cnt[kChkClasses];
    int fst[kChkClasses];
    const int rc = check_state(S, c, hc.t, cnt, fst);
    if (rc) return rc;
    for (int k = 0; k < kChkClasses; ++k) {
        counts[k] = (int64_t)cnt[k];
        if (first) first[k] = fst[k];
    }
    return SIM_OK;
}

int sim_read_emissions(sim_t* S, float* fuel, float* co) {
    if (!S) return SIM_EINVAL;
    if (!S->loaded || S->ntrips == 0) return SIM_OK;
    if (fuel)
        HIPCHECK(S, hipMemcpyAsync(fuel, S->tr.fuel_total, sizeof(float) * S->ntrips, hipMemcpyDeviceToHost, S->stream));
    if (co)
        HIPCHECK(S, hipMemcpyAsync(co, S->tr.co_total, sizeof(float) * S->ntrips, hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    return SIM_OK;
}

int sim_set_sampler(sim_t* S, int32_t every, int32_t group, int32_t max_groups) {
    if (!S || every <= 0 || group <= 0 || max_groups <= 0) return SIM_EINVAL;
    const size_t n = (size_t)max_groups * (size_t)S->ne;
    if (n > ((size_t)1 << 34)) return fail(S, SIM_EINVAL, "sampler too large");
    unsigned long long *cnt = nullptr, *spd = nullptr;
    if (!dalloc(S, cnt, n) || !dalloc(S, spd, n)) return fail(S, SIM_ENOMEM, "sampler allocation failed");
    HIPCHECK(S, hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * n, S->stream));
    HIPCHECK(S, hipMemsetAsync(spd, 0, sizeof(unsigned long long) * n, S->stream));
    S->s.samp_cnt = cnt;
    S->s.samp_spd = spd;
    S->s.samp_every = every;
    S->s.samp_group = group;
    S->s.samp_max = max_groups;
    drop_graphs(S);
    return SIM_OK;
}

int sim_read_samples(sim_t* S, int64_t* count, int64_t* speed_um) {
    if (!S) return SIM_EINVAL;
    if (S->s.samp_every <= 0) return fail(S, SIM_ESTATE, "no sampler");
    const size_t n = (size_t)S->s.samp_max * (size_t)S->ne;
    if (count) HIPCHECK(S, hipMemcpyAsync(count, S->s.samp_cnt, sizeof(int64_t) * n, hipMemcpyDeviceToHost, S->stream));
    if (speed_um)
        HIPCHECK(S, hipMemcpyAsync(speed_um, S->s.samp_spd, sizeof(int64_t) * n, hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    return SIM_OK;
}

int sim_set_idm(sim_t* S, const float* idm) {
    if (!S || !idm) return SIM_EINVAL;
    return upload_idm(S, idm);
}

int sim_set_vehicle_types(sim_t* S, int32_t num_types, const float* types, int32_t num_trips,
                          const uint8_t* trip_type) {
    if (!S || !types || num_types < 1 || num_types > 4 || num_trips < 0) return SIM_EINVAL;
    if (S->loaded) return fail(S, SIM_ESTATE, "vehicle types are set before the demand is loaded");
    for (int k = 0; k < num_types; ++k) {
        const float len = types[3 * k], am = types[3 * k + 1], vm = types[3 * k + 2];
        if (!(len > 0) || !std::isfinite(len) || !(am > 0) || !(vm > 0))
            return fail(S, SIM_EINVAL, "vehicle type " + std::to_string(k) + " out of range");
        for (int e = 0; e < S->ne; ++e)
            if (!((double)S->len[e] >= (double)len + (double)S->P.s0))
                return fail(S, SIM_EINVAL, "link " + std::to_string(e) + " is shorter than type " +
                                               std::to_string(k) + " plus the minimum gap");
    }
    for (int i = 0; i < num_trips; ++i)
        if (trip_type && trip_type[i] >= num_types) return fail(S, SIM_EINVAL, "trip type out of range");
    S->P.nt = num_types;
    S->tamax.assign(num_types, 0.0);
    S->tvmax.assign(num_types, 0.0);
    for (int k = 0; k < num_types; ++k) {
        S->P.tlen[k] = types[3 * k];
        S->P.tclaim[k] = (float)((double)types[3 * k] + (double)S->P.s0);
        S->tamax[k] = (double)types[3 * k + 1];
        S->tvmax[k] = (double)types[3 * k + 2];
    }
    S->trip_type.clear();
    if (trip_type) S->trip_type.assign(trip_type, trip_type + num_trips);
    S->typed = true;
    drop_graphs(S);
    const std::vector<float> idm = S->idm_in;
    return upload_idm(S, idm.data());
}

int sim_set_control(sim_t* S, const int32_t* node_control, int32_t signal_green_steps, float stop_dist,
                    float stop_speed) {
    if (!S || !node_control) return SIM_EINVAL;
    if (signal_green_steps <= 0 || !(stop_dist > 0) || !(stop_speed >= 0) || !std::isfinite(stop_dist) ||
        !std::isfinite(stop_speed))
        return fail(S, SIM_EINVAL, "invalid control parameters");
    if (S->tape_on) return fail(S, SIM_ESTATE, "control cannot change inside a differentiation window");
    std::vector<int> ctrl(node_control, node_control + S->nn);
    for (int u = 0; u < S->nn; ++u)
        if (ctrl[u] < 0 || ctrl[u] > 2) return fail(S, SIM_EINVAL, "node " + std::to_string(u) + ": control not 0, 1 or 2");
    // host sources stay alive until the stream is synchronised below
    std::vector<int> in_rank(S->ne), in_deg(S->nn, 0);
    if (!S->d_ctrl) {
        for (int e = 0; e < S->ne; ++e) in_rank[e] = in_deg[S->col_idx[e]]++;
        if (!dalloc(S, S->d_ctrl, S->nn) || !dalloc(S, S->d_in_rank, S->ne) || !dalloc(S, S->d_in_deg, S->nn))
            return fail(S, SIM_ENOMEM, "control allocation failed");
        int rc;
        if ((rc = h2d(S, S->d_in_rank, in_rank.data(), S->ne)) || (rc = h2d(S, S->d_in_deg, in_deg.data(), S->nn)))
            return rc;
    }
    int rc;
    if ((rc = h2d(S, S->d_ctrl, ctrl.data(), S->nn))) return rc;
    // every stop node starts free; requests are issued again from the current state
    const std::vector<int> none(S->nn, -1);
    if ((rc = h2d(S, S->s.holder, none.data(), S->nn))) return rc;
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(kBlock), 0, S->stream, S->s.stop_req, (long long)S->nn, ~0ull);
    S->P.green = signal_green_steps;
    S->P.stop_dist = stop_dist;
    S->P.stop_speed = stop_speed;
    S->net.ctrl = S->d_ctrl;
    S->net.in_rank = S->d_in_rank;
    S->net.in_deg = S->d_in_deg;
    drop_graphs(S);  // captured launches hold the old parameters
    if (S->loaded && (rc = reindex(S, S->buf[S->host_t & 1], S->s, S->ctr))) return rc;
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    return SIM_OK;
}

int sim_set_timing(sim_t* S, int32_t every) {
    if (!S || every < 0) return SIM_EINVAL;
    S->timing_every = every;
    return SIM_OK;
}

int sim_read_timing(sim_t* S, double* kernel_ms, int64_t* samples) {
    if (!S || !kernel_ms || !samples) return SIM_EINVAL;
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    for (auto& evs : S->ev_steps) {
        for (int q = 0; q < SIM_NUM_KERNELS; ++q) {
            float ms = 0.0f;
            HIPCHECK(S, hipEventElapsedTime(&ms, evs[2 * q], evs[2 * q + 1]));
            kernel_ms[q] += ms;
        }
        for (hipEvent_t e : evs) S->ev_free.push_back(e);
    }
    *samples = (int64_t)S->ev_steps.size();
    S->ev_steps.clear();
    return SIM_OK;
}

int sim_set_stream(sim_t* S, void* hip_stream) {
    if (!S) return SIM_EINVAL;
    HIPCHECK(S, S->stream ? hipStreamSynchronize(S->stream) : hipDeviceSynchronize());
    S->stream = static_cast<hipStream_t>(hip_stream);
    return SIM_OK;
}

void sim_destroy(sim_t* S) {
    if (!S) return;
    drop_graphs(S);
    if (S->gstream) {
        (void)hipStreamSynchronize(S->gstream);
        (void)hipStreamDestroy(S->gstream);
        (void)hipEventDestroy(S->gjoin[0]);
        (void)hipEventDestroy(S->gjoin[1]);
    }
    release_all(S);
    for (auto& evs : S->ev_steps)
        for (hipEvent_t e : evs) S->ev_free.push_back(e);
    for (hipEvent_t e : S->ev_free) (void)hipEventDestroy(e);
    delete S;
}


int sim_create_batch(int32_t n, const sim_network* nets, const sim_params* prms, void* hip_stream,
                     sim_alloc_fn alloc, sim_free_fn free_fn, void* alloc_ctx, sim_t** out) {
    if (n <= 0 || !nets || !prms || !out) return SIM_EINVAL;
    const sim_params& p0 = prms[0];
    std::vector<int32_t> row_ptr(1, 0), col_idx, lanes, cls;
    std::vector<float> len, speed, idm;
    std::vector<int> edge_off(1, 0);
    int node_off = 0, class_off = 0;
    for (int q = 0; q < n; ++q) {
        const sim_network& N = nets[q];
        const sim_params& P = prms[q];
        if (!N.row_ptr || !N.col_idx || !N.lanes || !N.length_m || !N.speed_mps || !P.idm || N.num_nodes <= 0 ||
            N.num_edges <= 0 || P.num_classes <= 0 || N.row_ptr[0] != 0 || N.row_ptr[N.num_nodes] != N.num_edges)
            return SIM_EINVAL;
        // everything but the car-following parameters is shared by the batch
        if (P.dt != p0.dt || P.veh_length != p0.veh_length || P.s0 != p0.s0 || P.s_eps != p0.s_eps ||
            P.b_max != p0.b_max || P.mobil_p != p0.mobil_p || P.mobil_athr != p0.mobil_athr ||
            P.mobil_bsafe != p0.mobil_bsafe || P.mand_dist != p0.mand_dist ||
            P.lc_cooldown_steps != p0.lc_cooldown_steps)
            return SIM_EINVAL;
        const int e0 = (int)col_idx.size();
        for (int u = 0; u < N.num_nodes; ++u) row_ptr.push_back(e0 + N.row_ptr[u + 1]);
        for (int e = 0; e < N.num_edges; ++e) {
            if (N.col_idx[e] < 0 || N.col_idx[e] >= N.num_nodes) return SIM_EINVAL;
            const int c = N.link_class ? N.link_class[e] : 0;
            if (c < 0 || c >= P.num_classes) return SIM_EINVAL;
            col_idx.push_back(N.col_idx[e] + node_off);
            lanes.push_back(N.lanes[e]);
            len.push_back(N.length_m[e]);
            speed.push_back(N.speed_mps[e]);
            cls.push_back(c + class_off);
        }
        idm.insert(idm.end(), P.idm, P.idm + 4 * (size_t)P.num_classes);
        node_off += N.num_nodes;
        class_off += P.num_classes;
        edge_off.push_back((int)col_idx.size());
        if ((long long)col_idx.size() > INT32_MAX / 2) return SIM_EINVAL;
    }
    sim_network net = {node_off, (int32_t)col_idx.size(), row_ptr.data(), col_idx.data(), lanes.data(), len.data(),
                       speed.data(), cls.data()};
    sim_params prm = p0;
    prm.num_classes = class_off;
    prm.idm = idm.data();
    int rc = sim_create(&net, &prm, hip_stream, alloc, free_fn, alloc_ctx, out);
    if (rc == SIM_OK) (*out)->batch_edge_off = edge_off;
    return rc;
}

int sim_load_demand_batch(sim_t* S, int32_t n, const int32_t* num_trips, const int32_t* const* depart_step,
                          const int32_t* const* trip_route, const int32_t* num_routes,
                          const int64_t* const* route_ptr, const int32_t* const* route_edges) {
    if (!S) return SIM_EINVAL;
    if ((int)S->batch_edge_off.size() != n + 1 || n <= 0)
        return fail(S, SIM_ESTATE, "handle was not created by sim_create_batch with this many scenarios");
    if (!num_trips || !depart_step || !trip_route || !num_routes || !route_ptr || !route_edges)
        return fail(S, SIM_EINVAL, "null batch demand arrays");
    std::vector<int32_t> dep, trt, re;
    std::vector<int64_t> rp(1, 0);
    int route_off = 0;
    for (int q = 0; q < n; ++q) {
        const int ne_q = S->batch_edge_off[q + 1] - S->batch_edge_off[q];
        if (num_trips[q] < 0 || num_routes[q] < 0 || !route_ptr[q] || route_ptr[q][0] != 0 ||
            (num_trips[q] > 0 && (!depart_step[q] || !trip_route[q] || num_routes[q] == 0)))
            return fail(S, SIM_EINVAL, "invalid demand of scenario " + std::to_string(q));
        for (int i = 0; i < num_trips[q]; ++i) {
            if (trip_route[q][i] < 0 || trip_route[q][i] >= num_routes[q])
                return fail(S, SIM_EINVAL, "trip_route out of range in scenario " + std::to_string(q));
            dep.push_back(depart_step[q][i]);
            trt.push_back(trip_route[q][i] + route_off);
        }
        const long long base = (long long)re.size();
        for (int r = 0; r < num_routes[q]; ++r) {
            for (long long k = route_ptr[q][r]; k < route_ptr[q][r + 1]; ++k) {
                const int e = route_edges[q][k];
                if (e < 0 || e >= ne_q) return fail(S, SIM_EROUTE, "edge id out of range in scenario " + std::to_string(q));
                re.push_back(e + S->batch_edge_off[q]);
            }
            rp.push_back(base + route_ptr[q][r + 1]);
        }
        route_off += num_routes[q];
        if ((long long)re.size() > INT32_MAX - 2) return fail(S, SIM_EROUTE, "route_edges too long");
    }
    return sim_load_demand(S, (int32_t)dep.size(), dep.data(), trt.data(), route_off, rp.data(), re.data(), nullptr,
                           nullptr, nullptr);
}

int sim_reload_routes(sim_t* S, const int64_t* route_ptr, const int32_t* route_edges, int64_t total_route_edges) {
    if (!S) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    if (S->placed) return fail(S, SIM_ESTATE, "the demand placed vehicles on the road: no route reload");
    if (!S->batch_edge_off.empty()) return fail(S, SIM_ESTATE, "no route reload on a batch of scenarios");
    if (S->tape_on || S->adj_ready) return fail(S, SIM_ESTATE, "no route reload inside a differentiation window");
    if (!route_ptr || total_route_edges < 0 || (total_route_edges > 0 && !route_edges))
        return fail(S, SIM_EINVAL, "null or negative route arrays");
    if (total_route_edges > (long long)INT32_MAX - 2) return fail(S, SIM_EROUTE, "route_edges too long");
    const int n = S->ntrips;
    const long long total = total_route_edges;
    long long last = -1;
    HIPCHECK(S, hipMemcpyAsync(&last, route_ptr + n, sizeof(long long), hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    if (last != total) return fail(S, SIM_EINVAL, "route_ptr[num_trips] differs from total_route_edges");
    if (!S->d_tail) {
        if (!dalloc(S, S->d_tail, (size_t)S->ne) || !dalloc(S, S->d_rkey, 2 * (size_t)S->cap) ||
            !dalloc(S, S->d_rval, 2 * (size_t)S->cap) || !dalloc(S, S->d_rerr, 2))
            return fail(S, SIM_ENOMEM, "route reload: scratch allocation failed");
        int rc = h2d(S, S->d_tail, S->tail.data(), (size_t)S->ne);
        if (rc) return rc;
    }
    const dim3 gn((unsigned)std::min<long long>(kMaxGrid, std::max<long long>(1, ((long long)n + kBlock - 1) / kBlock)));
    const dim3 b(kBlock);
    // every route checked before anything changes
    const int none = INT32_MAX;
    int bad = INT32_MAX;
    HIPCHECK(S, hipMemcpyAsync(S->d_rerr, &none, sizeof(int), hipMemcpyHostToDevice, S->stream));
    if (n > 0)
        hipLaunchKernelGGL(k_route_check, gn, b, 0, S->stream, route_ptr, route_edges, total, n, S->ne, S->net.head,
                           S->d_tail, S->d_rerr);
    HIPCHECK(S, hipGetLastError());
    HIPCHECK(S, hipMemcpyAsync(&bad, S->d_rerr, sizeof(int), hipMemcpyDeviceToHost, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    if (bad != INT32_MAX)
        return fail(S, SIM_EROUTE, "route of trip " + std::to_string(bad) + " is empty, out of range or not contiguous");

    // the route table, copied in
    drop_graphs(S);
    if (total > S->re_cap) {
        dfree(S, S->tr.route_edges);
        int* re = nullptr;
        if (!dalloc(S, re, (size_t)total)) return fail(S, SIM_ENOMEM, "route reload: route table allocation failed");
        S->tr.route_edges = re;
        S->re_cap = total;
    }
    int* re = const_cast<int*>(S->tr.route_edges);
    if (total > 0)
        HIPCHECK(S, hipMemcpyAsync(re, route_edges, sizeof(int) * (size_t)total, hipMemcpyDeviceToDevice, S->stream));
    // per vehicle id its route, and the departure queues: trips by (first
    // link, type), each queue by vehicle id (a stable sort of the ids by key)
    int* rbeg = const_cast<int*>(S->tr.rbeg);
    int* rend = const_cast<int*>(S->tr.rend);
    int* qvid = const_cast<int*>(S->tr.qvid);
    unsigned* key = S->d_rkey;
    unsigned* skey = S->d_rkey + S->cap;
    int* flag = S->d_rval;
    int* qidx = S->d_rval + S->cap;
    int nq = 0;
    if (n > 0) {
        hipLaunchKernelGGL(k_route_trips, gn, b, 0, S->stream, route_ptr, re, S->d_ord, S->d_vtype, n, rbeg, rend,
                           key, S->d_rval);
        HIPCHECK(S, hipGetLastError());
        unsigned bits = 1;
        while (bits < 32 && (1ull << bits) < 4ull * (unsigned long long)S->ne) ++bits;
        size_t b_sort = 0, b_scan = 0;
        HIPCHECK(S, rocprim::radix_sort_pairs(nullptr, b_sort, key, skey, S->d_rval, qvid, (size_t)n, 0, bits,
                                              S->stream));
        HIPCHECK(S, rocprim::exclusive_scan(nullptr, b_scan, flag, qidx, 0, (size_t)n, rocprim::plus<int>(),
                                            S->stream));
        const size_t need = std::max(b_sort, b_scan);
        if (need > S->rtmp_bytes) {
            dfree(S, S->d_rtmp);
            void* tmp = raw_alloc(S, need);
            if (!tmp) return fail(S, SIM_ENOMEM, "route reload: sort scratch allocation failed");
            S->d_rtmp = tmp;
            S->rtmp_bytes = need;
        }
        size_t bytes = S->rtmp_bytes;
        HIPCHECK(S, rocprim::radix_sort_pairs(S->d_rtmp, bytes, key, skey, S->d_rval, qvid, (size_t)n, 0, bits,
                                              S->stream));
        hipLaunchKernelGGL(k_queue_flags, gn, b, 0, S->stream, skey, n, flag);
        bytes = S->rtmp_bytes;
        HIPCHECK(S, rocprim::exclusive_scan(S->d_rtmp, bytes, flag, qidx, 0, (size_t)n, rocprim::plus<int>(),
                                            S->stream));
        hipLaunchKernelGGL(k_queue_count, dim3(1), dim3(64), 0, S->stream, flag, qidx, n, S->d_rerr + 1);
        HIPCHECK(S, hipGetLastError());
        HIPCHECK(S, hipMemcpyAsync(&nq, S->d_rerr + 1, sizeof(int), hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipStreamSynchronize(S->stream));
        int rc = grow_queues(S, nq);
        if (rc) return rc;
        hipLaunchKernelGGL(k_queue_build, gn, b, 0, S->stream, skey, qvid, flag, qidx, S->d_dep, n,
                           const_cast<int*>(S->tr.qoff), const_cast<int*>(S->tr.qedge),
                           const_cast<unsigned char*>(S->tr.qtype), const_cast<int*>(S->tr.qdep));
        HIPCHECK(S, hipGetLastError());
    }
    S->tr.nq = nq;
    S->tr.qhead = S->qstate;
    S->tr.qtail = S->qstate + nq;
    S->grid_q = (int)std::min<long long>(kMaxGrid, std::max<long long>(1, ((long long)nq + kBlock - 1) / kBlock));

    // the dynamic state back to the demand's first step: no vehicle on the
    // road, empty queues, statistics and trip outcomes
    Scratch& s = S->s;
    const size_t cap = (size_t)S->cap, ne = (size_t)S->ne;
    const dim3 gc((unsigned)std::min<size_t>(kMaxGrid, (cap + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_fill_i32, gc, b, 0, S->stream, S->tr.depart_actual, (long long)cap, -1);
    hipLaunchKernelGGL(k_fill_i32, gc, b, 0, S->stream, S->tr.arrive_step, (long long)cap, -1);
    hipLaunchKernelGGL(k_fill_i32, dim3(std::max(1, std::min(kMaxGrid, (S->nn + kBlock - 1) / kBlock))), b, 0,
                       S->stream, s.holder, (long long)S->nn, -1);
    HIPCHECK(S, hipGetLastError());
    HIPCHECK(S, hipMemsetAsync(S->tr.fuel_total, 0, sizeof(float) * cap, S->stream));
    HIPCHECK(S, hipMemsetAsync(S->tr.co_total, 0, sizeof(float) * cap, S->stream));
    if (nq) HIPCHECK(S, hipMemsetAsync(S->qstate, 0, sizeof(int) * 2 * (size_t)nq, S->stream));
    HIPCHECK(S, hipMemsetAsync(s.st_cnt, 0, sizeof(unsigned long long) * ne, S->stream));
    HIPCHECK(S, hipMemsetAsync(s.st_steps, 0, sizeof(unsigned long long) * ne, S->stream));
    HIPCHECK(S, hipMemsetAsync(s.st_us, 0, sizeof(unsigned long long) * ne, S->stream));
    if (s.samp_every > 0) {
        const size_t ns = (size_t)s.samp_max * ne;
        HIPCHECK(S, hipMemsetAsync(s.samp_cnt, 0, sizeof(unsigned long long) * ns, S->stream));
        HIPCHECK(S, hipMemsetAsync(s.samp_spd, 0, sizeof(unsigned long long) * ns, S->stream));
    }
    HIPCHECK(S, hipMemsetAsync(s.stay, 0, cap + 1, S->stream));
    HIPCHECK(S, hipMemsetAsync(s.mcnt, 0, sizeof(int) * (cap + 1), S->stream));
    HIPCHECK(S, hipMemsetAsync(s.ccnt, 0, sizeof(int) * 3 * kSeg * kSegStride, S->stream));
    HIPCHECK(S, hipMemsetAsync(s.sstat, 0, sizeof(unsigned long long) * kSeg * kStatStride, S->stream));
    Counters c0{};
    c0.t = (int)S->t_load;
    HIPCHECK(S, hipMemcpyAsync(S->ctr, &c0, sizeof(Counters), hipMemcpyHostToDevice, S->stream));
    S->host_t = S->t_load;
    int rc = reindex(S, S->buf[S->host_t & 1], S->s, S->ctr);
    if (rc) return rc;
    if (n > 0) HIPCHECK(S, hipMemcpyAsync(S->h_rbeg.data(), rbeg, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost,
                                          S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    return SIM_OK;
}

int sim_set_launch(sim_t* S, int32_t grid, int32_t grid_small) {
    if (!S || grid <= 0 || grid_small <= 0 || grid > 65536 || grid_small > 65536) return SIM_EINVAL;
    if (S->adj_ready) return fail(S, SIM_ESTATE, "launch shape is fixed once the adjoint buffers exist");
    S->grid = grid;
    S->grid_small = grid_small;
    drop_graphs(S);
    return SIM_OK;
}

int sim_get_launch(sim_t* S, int32_t* grid, int32_t* grid_small) {
    if (!S || !grid || !grid_small) return SIM_EINVAL;
    *grid = S->grid;
    *grid_small = S->grid_small;
    return SIM_OK;
}

int sim_set_decide_shape(sim_t* S, int32_t block, int32_t per_thread) {
    if (!S) return SIM_EINVAL;
    const int k = decide_shape_index(block, per_thread);
    if (k < 0) return fail(S, SIM_EINVAL, "no such decide shape");
    if (S->adj_ready) return fail(S, SIM_ESTATE, "launch shape is fixed once the adjoint buffers exist");
    if (k != S->dshape) drop_graphs(S);
    S->dshape = k;
    return SIM_OK;
}

int sim_get_decide_shape(sim_t* S, int32_t* block, int32_t* per_thread) {
    if (!S || !block || !per_thread) return SIM_EINVAL;
    *block = kDecideShapes[S->dshape].block;
    *per_thread = kDecideShapes[S->dshape].per;
    return SIM_OK;
}

int sim_step_graph(sim_t* S, int32_t num_steps, int32_t chunk) {
    if (!S || num_steps < 0 || chunk <= 0) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    if (S->tape_on) return sim_step(S, num_steps);  // checkpoints are per-step host work: no capture
    int done = 0;
    for (;;) {
        // with timing on, every timing_every-th step runs alone (timed) and the
        // steps between are replayed from graphs of that length
        int len = chunk;
        if (S->timing_every > 0) {
            const int to_timed = (int)(S->timing_every - (S->host_t % S->timing_every));
            if (to_timed == S->timing_every) {
                if (done >= num_steps) break;
                int rc = sim_step(S, 1);
                if (rc) return rc;
                done += 1;
                continue;
            }
            len = std::min(chunk, to_timed);
        }
        if (num_steps - done < len) break;
        if (len < 2) {  // one step before the next timed one: no graph for it
            int rc = sim_step(S, 1);
            if (rc) return rc;
            done += 1;
            continue;
        }
        int rc0 = graph_stream(S);
        if (rc0) return rc0;
        const int parity = (int)(S->host_t & 1);
        hipGraphExec_t exec = nullptr;
        for (auto& g : S->graphs)
            if (g.parity == parity && g.chunk == len) exec = g.exec;
        if (!exec) {
            if (S->graphs.size() >= 8) drop_graphs(S);
            hipGraph_t graph;
            HIPCHECK(S, hipStreamBeginCapture(S->gstream, hipStreamCaptureModeThreadLocal));
            const Tape off{};
            int rc = SIM_OK;
            hipStream_t user = S->stream;
            S->stream = S->gstream;  // launch_step enqueues on S->stream
            for (int k = 0; k < len && rc == SIM_OK; ++k) {
                const int p = (parity + k) & 1;
                rc = launch_step(S, S->buf[p], S->buf[p ^ 1], S->tr, S->s, off, S->ctr, nullptr);
            }
            S->stream = user;
            hipError_t ce = hipStreamEndCapture(S->gstream, &graph);
            if (rc) {
                if (ce == hipSuccess) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                return rc;
            }
            if (ce != hipSuccess) {
                (void)hipGetLastError();
                return fail(S, SIM_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
            }
            ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ce != hipSuccess) {
                (void)hipGetLastError();
                return fail(S, SIM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ce));
            }
            sim_t::GraphEntry ge;
            ge.parity = parity;
            ge.chunk = len;
            ge.exec = exec;
            S->graphs.push_back(ge);
        }
        HIPCHECK(S, hipEventRecord(S->gjoin[0], S->stream));
        HIPCHECK(S, hipStreamWaitEvent(S->gstream, S->gjoin[0], 0));
        HIPCHECK(S, hipGraphLaunch(exec, S->gstream));
        HIPCHECK(S, hipEventRecord(S->gjoin[1], S->gstream));
        HIPCHECK(S, hipStreamWaitEvent(S->stream, S->gjoin[1], 0));
        S->host_t += len;
        done += len;
    }
    return sim_step(S, num_steps - done);
}

void release_from(sim_t* S, size_t mark) {
    if (S->allocs.size() <= mark) return;
    (void)hipStreamSynchronize(S->stream);
    for (size_t k = mark; k < S->allocs.size(); ++k) {
        if (S->free_fn) S->free_fn(S->ctx, S->allocs[k]);
        else (void)hipFree(S->allocs[k]);
    }
    S->allocs.resize(mark);
}

int sim_autotune(sim_t* S, int32_t steps_per_trial, int32_t* best_grid, int32_t* best_small, float* best_ms) {
    if (!S || steps_per_trial <= 0 || !best_grid || !best_small || !best_ms) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    if (S->tape_on || S->adj_ready) return fail(S, SIM_ESTATE, "no tuning inside a differentiation window");
    // save the state and the statistics, try every candidate from the same
    // state, restore; the step's results do not depend on the launch shape.
    // The saved copy is freed on return, and every exit, error or not, puts
    // back the state, the statistics, the sampler and a launch shape.
    const size_t mark = S->allocs.size();
    sim_t::Ckpt save;
    const int p = (int)(S->host_t & 1);
    unsigned long long* st_save = nullptr;
    int* trip_save = nullptr;
    if (!alloc_veh(S, save.v, S->cap) || !alloc_cold(S, save.c, S->cap) || !dalloc(S, save.qstate, 2 * (size_t)S->tr.nq) ||
        !dalloc(S, save.ctr, 1) ||
        !dalloc(S, st_save, 3 * (size_t)S->ne) || !dalloc(S, trip_save, 4 * (size_t)S->cap) ||
        !dalloc(S, save.holder, S->nn)) {
        release_from(S, mark);
        return fail(S, SIM_ENOMEM, "autotune allocation failed");
    }
    const size_t tb = sizeof(int) * (size_t)S->cap;
    const size_t eb = sizeof(unsigned long long) * (size_t)S->ne;
    const long long t_save = S->host_t;
    const int samp_every = S->s.samp_every;
    int bg = S->grid, bs = S->grid_small, bd = S->dshape;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool saved = false;
    // put the saved state back (after every trial, and at the end)
    auto restore_state = [&]() -> int {
        S->host_t = t_save;
        int r = copy_state(S, S->buf[p], cold_of(S->tr), S->qstate, S->ctr, S->s.holder, save.v, save.c, save.qstate,
                           save.ctr, save.holder);
        if (r) return r;
        return reindex(S, S->buf[p], S->s, S->ctr);
    };
    auto finish = [&](int rc) -> int {
        S->s.samp_every = samp_every;
        S->grid = bg;
        S->grid_small = bs;
        S->dshape = bd;
        drop_graphs(S);
        if (saved) {
            int r = restore_state();
            hipError_t he = hipSuccess;
            he = hipMemcpyAsync(S->s.st_cnt, st_save, eb, hipMemcpyDeviceToDevice, S->stream);
            if (he == hipSuccess) he = hipMemcpyAsync(S->s.st_steps, st_save + S->ne, eb, hipMemcpyDeviceToDevice, S->stream);
            if (he == hipSuccess) he = hipMemcpyAsync(S->s.st_us, st_save + 2 * (size_t)S->ne, eb, hipMemcpyDeviceToDevice, S->stream);
            if (he == hipSuccess) he = hipMemcpyAsync(S->tr.depart_actual, trip_save, tb, hipMemcpyDeviceToDevice, S->stream);
            if (he == hipSuccess) he = hipMemcpyAsync(S->tr.arrive_step, trip_save + S->cap, tb, hipMemcpyDeviceToDevice, S->stream);
            if (he == hipSuccess) he = hipMemcpyAsync(S->tr.fuel_total, trip_save + 2 * (size_t)S->cap, tb, hipMemcpyDeviceToDevice, S->stream);
            if (he == hipSuccess) he = hipMemcpyAsync(S->tr.co_total, trip_save + 3 * (size_t)S->cap, tb, hipMemcpyDeviceToDevice, S->stream);
            if (he == hipSuccess) he = hipStreamSynchronize(S->stream);
            if (he != hipSuccess) {
                (void)hipGetLastError();
                if (!rc) rc = fail(S, SIM_EHIP, std::string("autotune restore: ") + hipGetErrorString(he));
            }
            if (!rc) rc = r;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        release_from(S, mark);
        return rc;
    };
#define TUNE_CHECK(call)                                                                            \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            (void)hipGetLastError();                                                                \
            return finish(fail(S, SIM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)));    \
        }                                                                                           \
    } while (0)
    TUNE_CHECK(hipMemcpyAsync(trip_save, S->tr.depart_actual, tb, hipMemcpyDeviceToDevice, S->stream));
    TUNE_CHECK(hipMemcpyAsync(trip_save + S->cap, S->tr.arrive_step, tb, hipMemcpyDeviceToDevice, S->stream));
    TUNE_CHECK(hipMemcpyAsync(trip_save + 2 * (size_t)S->cap, S->tr.fuel_total, tb, hipMemcpyDeviceToDevice, S->stream));
    TUNE_CHECK(hipMemcpyAsync(trip_save + 3 * (size_t)S->cap, S->tr.co_total, tb, hipMemcpyDeviceToDevice, S->stream));
    int rc = copy_state(S, save.v, save.c, save.qstate, save.ctr, save.holder, S->buf[p], cold_of(S->tr), S->qstate,
                        S->ctr, S->s.holder);
    if (rc) return finish(rc);
    TUNE_CHECK(hipMemcpyAsync(st_save, S->s.st_cnt, eb, hipMemcpyDeviceToDevice, S->stream));
    TUNE_CHECK(hipMemcpyAsync(st_save + S->ne, S->s.st_steps, eb, hipMemcpyDeviceToDevice, S->stream));
    TUNE_CHECK(hipMemcpyAsync(st_save + 2 * (size_t)S->ne, S->s.st_us, eb, hipMemcpyDeviceToDevice, S->stream));
    saved = true;
    TUNE_CHECK(hipEventCreate(&e0));
    TUNE_CHECK(hipEventCreate(&e1));
    S->s.samp_every = 0;  // trials take no samples
    const Tape off{};
    float best = 1e30f;
    // one trial: steps_per_trial steps of the given shape from the saved state
    auto trial = [&](int gc, int gs, int ds, float* ms) -> int {
        S->grid = gc;
        S->grid_small = gs;
        S->dshape = ds;
        int r = restore_state();
        if (r) return r;
        hipError_t he = hipEventRecord(e0, S->stream);
        for (int k = 0; k < steps_per_trial && r == SIM_OK && he == hipSuccess; ++k) {
            const int q = (int)(S->host_t & 1);
            r = launch_step(S, S->buf[q], S->buf[q ^ 1], S->tr, S->s, off, S->ctr, nullptr);
            S->host_t += 1;
        }
        if (r) return r;
        if (he == hipSuccess) he = hipEventRecord(e1, S->stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(ms, e0, e1);
        if (he != hipSuccess) {
            (void)hipGetLastError();
            return fail(S, SIM_EHIP, std::string("autotune trial: ") + hipGetErrorString(he));
        }
        return SIM_OK;
    };
    // grid counts and k_scan's share of them with the current decide shape,
    // then the decide shapes with the best grids; each candidate twice, a
    // shape's time is the faster of its trials
    const int g0 = S->grid;
    const int gcand[] = {g0 / 4, g0 / 2, g0 * 3 / 4, g0, g0 * 3 / 2, g0 * 2};
    for (int pass = 0; pass < 2; ++pass)
        for (int gc : gcand) {
            if (gc < 1) continue;
            // the scan's blocks: a share of the grid, or a fixed few (its
            // tiles are taken from a counter, and fewer blocks contend less)
            int scand[5] = {gc / 2, gc / 4, gc / 8, 128, 256};
            for (int c = 0; c < 5; ++c) {
                const int gs = std::max(1, std::min(gc, scand[c]));
                bool seen = false;
                for (int c2 = 0; c2 < c; ++c2) seen |= std::max(1, std::min(gc, scand[c2])) == gs;
                if (seen) continue;
                float ms = 0.0f;
                if ((rc = trial(gc, gs, bd, &ms))) return finish(rc);
                if (ms < best) {
                    best = ms;
                    bg = gc;
                    bs = gs;
                }
            }
        }
    const int dcur = bd, g1 = bg, s1 = bs;
    for (int pass = 0; pass < 2; ++pass)
        for (int ds = 0; ds < kNumDecideShapes; ++ds) {
            if (ds == dcur) continue;
            for (int gc : {g1 / 2, g1, g1 * 2}) {
                if (gc < 1) continue;
                const int gs = std::max(1, (int)((long long)s1 * gc / g1));
                float ms = 0.0f;
                if ((rc = trial(gc, gs, ds, &ms))) return finish(rc);
                if (ms < best) {
                    best = ms;
                    bd = ds;
                    bg = gc;
                    bs = gs;
                }
            }
        }
#undef TUNE_CHECK
    rc = finish(SIM_OK);
    if (rc) return rc;
    *best_grid = bg;
    *best_small = bs;
    *best_ms = best / (float)steps_per_trial;
    return SIM_OK;
}

}  // extern "C"
