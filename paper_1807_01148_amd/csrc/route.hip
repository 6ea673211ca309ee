// Route planning for iterative re-routing (Sec. 6.3.1) on MI355X: the C ABI
// of include/trafficroute.h.
//
// Shortest paths from many origins at once.  For a batch of B origins the
// labels live in one array key[b * nn + v] of 64-bit words
//     (distance in ms) << 24 | (last edge of the route)
// so a single 64-bit atomicMin both lowers the distance and, among equal
// distances, keeps the lowest-numbered tight edge: the route rule of the
// header falls out of the integer order of the words, whatever the order in
// which relaxations land.  The search is a frontier Bellman-Ford: a round
// relaxes the out-edges of every (origin, node) whose distance dropped in the
// round before (a per-label round stamp keeps each label at most once in a
// frontier).  Integer weights make the result exact and order-free.
//
// To keep the work near that of Dijkstra the rounds are banded (a near/far
// split of delta-stepping): a label that drops below the current threshold T
// joins the next round's frontier, one that drops to T or more waits in a far
// list; when the frontier runs dry T grows by delta and the far labels below
// it form the next frontier.  Any order of relaxations ends at the same
// labels, so the banding changes the work, never the result.
//
// Routes of the selected trips are read back from the predecessor arrays of
// their origins (count, scan, write from the destination backwards); the
// other trips' routes are copied.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "trafficroute.h"

namespace troute {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kEdgeBits = 24;
constexpr unsigned long long kEdgeMask = (1ull << kEdgeBits) - 1ull;  // also "no edge" (the origin)
constexpr unsigned long long kUnreached = ~0ull;
constexpr int kMaxGrid = 8192;
constexpr int kScanTile = 2048;  // entries per block in the route-length scan
constexpr int kRoundsPerCheck = 4;
constexpr int kRelaxMaxGrid = 16384;
constexpr int kMaxBatch = 4096;  // origins per search batch

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// consecutive slots for the lanes of a wave that reach this point together,
// with one atomic on the shared counter
__device__ __forceinline__ unsigned wave_slot(unsigned* counter) {
    const unsigned long long mask = __ballot(1);
    const int lane = (int)__lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    const unsigned rank = (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned)__popcll(mask));
    base = __shfl(base, leader, kWave);
    return base + rank;
}

__global__ void k_fill_keys(unsigned long long* key, unsigned* stamp, unsigned* fstamp, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        key[i] = kUnreached;
        stamp[i] = 0u;
        fstamp[i] = 0u;
    }
}

// counters of a search cleared by a kernel (no memset nodes in the stream):
// the five frontier and far-list counts (if cnt) and the first 64-bit word
__global__ void k_clear_counters(unsigned* cnt, unsigned long long* u64) {
    if (blockIdx.x == 0 && threadIdx.x < 5 && cnt) cnt[threadIdx.x] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0 && u64) u64[0] = 0ull;
}

__global__ void k_zero_u32(unsigned* p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = 0u;
}

// origin b of the batch: distance 0, no edge; it forms the first frontier
__global__ void k_seed(unsigned long long* key, const int* origins, int B, long long nn, unsigned* fr,
                       unsigned* cnt) {
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b < B) {
        const long long i = (long long)b * nn + origins[b];
        key[i] = kEdgeMask;
        fr[b] = (unsigned)i;
    }
    if (b == 0) {
        cnt[0] = (unsigned)B;
        cnt[1] = 0u;
        cnt[2] = 0u;
    }
}

// round r (from 0): relax the out-edges of the cnt[r % 3] entries of fin;
// labels that drop join fout (count cnt[(r + 1) % 3]), each at most once per
// round by its stamp r + 1; cnt[(r + 2) % 3], the input count of round
// r - 1, is cleared for round r + 1
// Labels that drop to thr or more go to the far list instead (each at most
// once per band, by its far stamp = the band number).
__global__ __launch_bounds__(kBlock) void k_relax(const int* __restrict__ row_ptr, const int* __restrict__ col,
                                                  const long long* __restrict__ w, unsigned long long* key,
                                                  unsigned* stamp, long long nn, const unsigned* __restrict__ fin,
                                                  unsigned* fout, unsigned* cnt, int r, unsigned long long* work,
                                                  unsigned long long thr, unsigned* fstamp, unsigned band,
                                                  unsigned* far, unsigned* nfar) {
    const unsigned nin = cnt[r % 3];
    unsigned* nout = cnt + (r + 1) % 3;
    const unsigned mark = (unsigned)r + 1u;
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[(r + 2) % 3] = 0u;
    unsigned long long done = 0;
    for (unsigned long long q = blockIdx.x * kBlock + threadIdx.x; q < nin; q += gridDim.x * kBlock) {
        const unsigned long long i = fin[q];
        const long long u = (long long)(i % (unsigned long long)nn);
        const unsigned long long base = i - (unsigned long long)u;
        const unsigned long long d = key[i] >> kEdgeBits;
        const int e0 = row_ptr[u], e1 = row_ptr[u + 1];
        for (int e = e0; e < e1; ++e) {
            const unsigned long long x = base + (unsigned long long)col[e];
            const unsigned long long nd = d + (unsigned long long)w[e];
            const unsigned long long old = atomicMin(key + x, (nd << kEdgeBits) | (unsigned long long)e);
            if (nd < (old >> kEdgeBits)) {
                if (nd < thr) {
                    if (atomicExch(stamp + x, mark) != mark) fout[wave_slot(nout)] = (unsigned)x;
                } else if (atomicExch(fstamp + x, band) != band) {
                    far[wave_slot(nfar)] = (unsigned)x;
                }
            }
        }
        done += (unsigned long long)(e1 - e0);
    }
    done = wave_sum(done);
    if ((threadIdx.x & (kWave - 1)) == 0 && done) atomicAdd(work, done);
}

// A new band [.., thr): far labels below thr form the frontier of round r
// (stamp r, as if pushed by round r - 1); the others stay far, stamped with
// the new band.  Stale entries (labels that dropped again since) are harmless.
__global__ void k_split(const unsigned long long* key, unsigned* stamp, unsigned* fstamp, const unsigned* far_in,
                        const unsigned* nfar_in, unsigned long long thr, unsigned band, unsigned* fr, unsigned* cnt,
                        int r, unsigned* far_out, unsigned* nfar_out) {
    const unsigned n = *nfar_in;
    unsigned* nnear = cnt + r % 3;
    for (unsigned long long q = blockIdx.x * kBlock + threadIdx.x; q < n; q += gridDim.x * kBlock) {
        const unsigned i = far_in[q];
        if ((key[i] >> kEdgeBits) < thr) {
            if (atomicExch(stamp + i, (unsigned)r) != (unsigned)r) fr[wave_slot(nnear)] = i;
        } else if (atomicExch(fstamp + i, band) != band) {
            far_out[wave_slot(nfar_out)] = i;
        }
    }
}

// predecessor edge per node of each origin of the batch (-1: origin, unreached)
__global__ void k_preds(const unsigned long long* key, long long n, int* pred) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const unsigned long long k = key[i];
        const unsigned long long e = k & kEdgeMask;
        pred[i] = (k == kUnreached || e == kEdgeMask) ? -1 : (int)e;
    }
}

__global__ void k_dists(const unsigned long long* key, long long n, long long* dist) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const unsigned long long k = key[i];
        dist[i] = k == kUnreached ? INT64_MAX : (long long)(k >> kEdgeBits);
    }
}

__global__ void k_weights_from_stats(const long long* cnt, const long long* tt_us, long long* w, int ne) {
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < ne; e += gridDim.x * kBlock) {
        const long long c = cnt[e];
        if (c > 0) {
            const long long m = (tt_us[e] + 500 * c) / (1000 * c);
            w[e] = m < 1 ? 1 : m;
        }
    }
}

__global__ void k_weight_sum(const long long* w, int ne, unsigned long long* out) {
    unsigned long long s = 0;
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < ne; e += gridDim.x * kBlock) s += (unsigned long long)w[e];
    s = wave_sum(s);
    if ((threadIdx.x & (kWave - 1)) == 0 && s) atomicAdd(out, s);
}

struct TripView {
    const int* src;     // origin index per trip
    const int* dst;     // destination node per trip
    const int* origin;  // node of each origin index
    const int* pred;    // [num origins][nn]
    const int* tail;
    long long nn;
    int n;
    const unsigned char* sel;  // null: every trip
};

// route length of every trip (selected: walk the predecessor edges back from
// the destination; others: the current length)
__global__ void k_route_len(TripView T, const long long* old_ptr, long long* len, unsigned* err) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < T.n; i += gridDim.x * kBlock) {
        if (T.sel && !T.sel[i]) {
            len[i] = old_ptr[i + 1] - old_ptr[i];
            continue;
        }
        const int s = T.src[i];
        const int o = T.origin[s];
        const int* P = T.pred + (long long)s * T.nn;
        int v = T.dst[i];
        long long n = 0;
        while (v != o) {
            const int e = P[v];
            if (e < 0 || n >= T.nn) {  // unreachable (or a broken tree): flag it
                atomicOr(err, 1u);
                n = 0;
                break;
            }
            v = T.tail[e];
            ++n;
        }
        if (n == 0) atomicOr(err, 1u);  // also: destination == origin
        len[i] = n;
    }
}

__global__ void k_route_write(TripView T, const long long* old_ptr, const int* old_edges, const long long* ptr,
                              int* edges) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < T.n; i += gridDim.x * kBlock) {
        if (T.sel && !T.sel[i]) {
            const long long a = old_ptr[i], n = old_ptr[i + 1] - a, b = ptr[i];
            for (long long k = 0; k < n; ++k) edges[b + k] = old_edges[a + k];
            continue;
        }
        const int s = T.src[i];
        const int o = T.origin[s];
        const int* P = T.pred + (long long)s * T.nn;
        int v = T.dst[i];
        long long pos = ptr[i + 1] - 1;
        while (v != o && pos >= ptr[i]) {  // the length pass walked this route already
            const int e = P[v];
            edges[pos--] = e;
            v = T.tail[e];
        }
    }
}

// inclusive scan of len into ptr[1..n] (ptr[0] = 0): tile sums, a scan of the
// tile sums in one block, then each tile scanned with its offset
__global__ void k_tile_sums(const long long* len, int n, long long* tsum) {
    __shared__ long long red[kBlock];
    const long long t0 = (long long)blockIdx.x * kScanTile;
    long long s = 0;
    for (int k = threadIdx.x; k < kScanTile; k += kBlock)
        if (t0 + k < n) s += len[t0 + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) tsum[blockIdx.x] = red[0];
}

__global__ void k_scan_tiles(long long* tsum, int ntiles) {
    // one block; exclusive scan in chunks of kBlock with a running carry
    __shared__ long long buf[kBlock];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < ntiles; c0 += kBlock) {
        const int i = c0 + threadIdx.x;
        const long long v = i < ntiles ? tsum[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kBlock; o <<= 1) {
            long long y = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < ntiles) tsum[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry += buf[kBlock - 1];
        __syncthreads();
    }
}

__global__ void k_tile_apply(const long long* len, int n, const long long* toff, long long* ptr) {
    __shared__ long long buf[kBlock];
    const long long t0 = (long long)blockIdx.x * kScanTile;
    constexpr int kPer = kScanTile / kBlock;
    long long v[kPer];
    long long s = 0;
    for (int k = 0; k < kPer; ++k) {
        const long long i = t0 + (long long)threadIdx.x * kPer + k;
        v[k] = i < n ? len[i] : 0;
        s += v[k];
    }
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        long long y = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
        __syncthreads();
        buf[threadIdx.x] += y;
        __syncthreads();
    }
    long long run = toff[blockIdx.x] + buf[threadIdx.x] - s;
    for (int k = 0; k < kPer; ++k) {
        const long long i = t0 + (long long)threadIdx.x * kPer + k;
        run += v[k];
        if (i < n) ptr[i + 1] = run;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ptr[0] = 0;
}

}  // namespace troute

using namespace troute;

struct rt_t {
    int device = 0;  // current device at rt_create
    hipStream_t stream = nullptr;
    sim_alloc_fn alloc = nullptr;
    sim_free_fn free_fn = nullptr;
    void* ctx = nullptr;
    std::string err;
    std::vector<void*> allocs;

    int nn = 0, ne = 0;
    std::vector<int> row_ptr, col_idx, lanes;
    std::vector<float> len, speed;
    int* d_row_ptr = nullptr;
    int* d_col = nullptr;
    int* d_tail = nullptr;
    long long* d_w = nullptr;
    unsigned long long* d_u64 = nullptr;  // [0] relaxations, [1] weight sum
    unsigned* d_err = nullptr;
    unsigned* d_cnt = nullptr;  // three rotating frontier counters, two far-list counters

    // trips
    int nsrc = 0, ntrips = 0;
    std::vector<int> h_src_nodes, h_trip_src;
    int* d_src_nodes = nullptr;
    int* d_trip_src = nullptr;
    int* d_trip_dst = nullptr;
    int* d_pred = nullptr;  // [nsrc][nn]
    unsigned char* d_sel = nullptr;
    long long* d_len = nullptr;
    long long* d_tsum = nullptr;

    // current routes
    bool have_routes = false;
    long long total = 0;
    long long* d_ptr = nullptr;
    int* d_edges = nullptr;

    // search batch
    int batch = 0;  // origins per batch; 0 = automatic
    int batch_alloc = 0;
    unsigned long long* d_key = nullptr;
    unsigned* d_stamp = nullptr;
    unsigned* d_fstamp = nullptr;
    unsigned* d_fr[2] = {nullptr, nullptr};
    unsigned* d_far[2] = {nullptr, nullptr};
    long long delta = 0;  // band width in ms; 0 = three times the mean weight
    long long wsum = 0;   // sum of the weights (checked before every search)
    int* d_origins = nullptr;

    long long last_relax = 0;
    int last_sources = 0;
};

namespace {

int rfail(rt_t* R, int code, const std::string& msg) {
    if (R) R->err = msg;
    return code;
}

#define RCHECK(R, call)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (void)hipGetLastError();                                                             \
            return rfail((R), SIM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
        }                                                                                        \
    } while (0)

void* ralloc(rt_t* R, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (R->alloc) {
        p = R->alloc(R->ctx, bytes);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p) R->allocs.push_back(p);
    return p;
}

void rfree(rt_t* R, void* p) {
    if (!p) return;
    auto it = std::find(R->allocs.begin(), R->allocs.end(), p);
    if (it == R->allocs.end()) return;
    R->allocs.erase(it);
    if (R->free_fn) R->free_fn(R->ctx, p);
    else (void)hipFree(p);
}

template <class T>
bool ra(rt_t* R, T*& out, size_t n) {
    out = static_cast<T*>(ralloc(R, sizeof(T) * (n ? n : 1)));
    return out != nullptr;
}

template <class T>
int rh2d(rt_t* R, T* dst, const T* src, size_t n) {
    if (n == 0) return SIM_OK;
    RCHECK(R, hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyHostToDevice, R->stream));
    return SIM_OK;
}

int grid_for(long long n) {
    return (int)std::min<long long>(kMaxGrid, std::max<long long>(1, (n + kBlock - 1) / kBlock));
}

int auto_batch(const rt_t* R) {
    // key (8 B) + two stamps (8 B) + two frontier and two far entries (16 B)
    // per (origin, node), within a quarter of the free device memory and at
    // most 64 GiB: the more origins per batch, the fewer rounds per plan (the
    // rounds of a batch follow the depth of the graph, not the origin count)
    const long long per = 32ll * R->nn;
    size_t free_b = 0, total_b = 0;
    long long budget = 4ll << 30;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
        budget = std::max<long long>(budget, std::min<long long>((long long)(free_b / 4), 64ll << 30));
    long long b = budget / std::max<long long>(per, 1);
    b = std::min<long long>(b, (long long)(UINT32_MAX / (unsigned long long)R->nn));
    return (int)std::max<long long>(1, std::min<long long>(b, kMaxBatch));
}

// blocks for a relaxation round whose frontier was last seen at est entries:
// room for four times that (it grows between checks); larger frontiers loop
int relax_grid(unsigned long long est) {
    const unsigned long long t = (4ull * std::max<unsigned long long>(est, 1ull) + kBlock - 1) / kBlock;
    return (int)std::min<unsigned long long>(t, (unsigned long long)kRelaxMaxGrid);
}

int ensure_batch(rt_t* R, int B) {
    if (B <= R->batch_alloc) return SIM_OK;
    for (void* p : {(void*)R->d_key, (void*)R->d_stamp, (void*)R->d_fstamp, (void*)R->d_fr[0], (void*)R->d_fr[1],
                    (void*)R->d_far[0], (void*)R->d_far[1]})
        rfree(R, p);
    rfree(R, R->d_origins);
    R->d_key = nullptr;
    R->d_stamp = R->d_fstamp = nullptr;
    R->d_fr[0] = R->d_fr[1] = R->d_far[0] = R->d_far[1] = nullptr;
    R->d_origins = nullptr;
    R->batch_alloc = 0;
    const size_t n = (size_t)B * (size_t)R->nn;
    if (!ra(R, R->d_key, n) || !ra(R, R->d_stamp, n) || !ra(R, R->d_fstamp, n) || !ra(R, R->d_fr[0], n) ||
        !ra(R, R->d_fr[1], n) || !ra(R, R->d_far[0], n) || !ra(R, R->d_far[1], n) || !ra(R, R->d_origins, (size_t)B))
        return rfail(R, SIM_ENOMEM, "search batch of " + std::to_string(B) + " origins does not fit");
    R->batch_alloc = B;
    return SIM_OK;
}

// The buffers of one search: per (origin, node) the label, the two stamps, two
// frontier and two far-list entries; the origins; five counters (three
// rotating frontier counts, two far-list counts) and two 64-bit words
// (relaxations, weight sum).
struct SearchBufs {
    unsigned long long* key;
    unsigned* stamp;
    unsigned* fstamp;
    unsigned* fr[2];
    unsigned* far[2];
    int* origins;
    unsigned* cnt;
    unsigned long long* u64;
};

SearchBufs handle_bufs(rt_t* R) {
    return SearchBufs{R->d_key, R->d_stamp, R->d_fstamp, {R->d_fr[0], R->d_fr[1]}, {R->d_far[0], R->d_far[1]},
                      R->d_origins, R->d_cnt, R->d_u64};
}

// shortest-path labels of the B origins already in b.origins, in b.key;
// adds the relaxations to *relax
int search_in(rt_t* R, const SearchBufs& b, int B, unsigned long long* relax) {
    const long long n = (long long)B * R->nn;
    hipLaunchKernelGGL(k_fill_keys, dim3(grid_for(n)), dim3(kBlock), 0, R->stream, b.key, b.stamp, b.fstamp, n);
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(kWave), 0, R->stream, b.cnt, b.u64);
    hipLaunchKernelGGL(k_seed, dim3((B + kBlock - 1) / kBlock), dim3(kBlock), 0, R->stream, b.key, b.origins, B,
                       (long long)R->nn, b.fr[0], b.cnt);
    RCHECK(R, hipGetLastError());
    const long long delta = R->delta > 0 ? R->delta : std::max<long long>(1, 3 * R->wsum / std::max(R->ne, 1));
    unsigned long long thr = (unsigned long long)delta;
    unsigned band = 1;
    unsigned long long est = (unsigned long long)B;  // frontier size last seen (the seeds)
    int r = 0;
    long long launched = 0;
    for (;;) {
        // rounds of the current band until its frontier runs dry
        unsigned c[5];
        for (;;) {
            const int g = relax_grid(est);
            for (int k = 0; k < kRoundsPerCheck; ++k, ++r) {
                hipLaunchKernelGGL(k_relax, dim3(g), dim3(kBlock), 0, R->stream, R->d_row_ptr, R->d_col, R->d_w,
                                   b.key, b.stamp, (long long)R->nn, b.fr[r & 1], b.fr[(r + 1) & 1], b.cnt, r, b.u64,
                                   thr, b.fstamp, band, b.far[band & 1], b.cnt + 3 + (band & 1));
            }
            RCHECK(R, hipGetLastError());
            RCHECK(R, hipMemcpyAsync(c, b.cnt, sizeof(c), hipMemcpyDeviceToHost, R->stream));
            RCHECK(R, hipStreamSynchronize(R->stream));
            launched += kRoundsPerCheck;
            if (c[r % 3] == 0) break;  // the frontier the next round would read
            est = c[r % 3];
            if (launched > 64ll * R->nn + 1024) return rfail(R, SIM_EHIP, "search did not converge");
        }
        if (c[3 + (band & 1)] == 0) break;  // nothing waits: every label is final
        // next band: far labels below the new threshold start the next round
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kWave), 0, R->stream, b.cnt + 3 + ((band + 1) & 1));
        thr += (unsigned long long)delta;
        hipLaunchKernelGGL(k_split, dim3(grid_for(c[3 + (band & 1)])), dim3(kBlock), 0, R->stream, b.key, b.stamp,
                           b.fstamp, b.far[band & 1], b.cnt + 3 + (band & 1), thr, band + 1, b.fr[r & 1], b.cnt, r,
                           b.far[(band + 1) & 1], b.cnt + 3 + ((band + 1) & 1));
        RCHECK(R, hipGetLastError());
        est = c[3 + (band & 1)];  // the new frontier is part of the far list
        ++band;
    }
    unsigned long long w = 0;
    RCHECK(R, hipMemcpyAsync(&w, b.u64, sizeof(w), hipMemcpyDeviceToHost, R->stream));
    RCHECK(R, hipStreamSynchronize(R->stream));
    *relax += w;
    return SIM_OK;
}

// shortest-path labels of origins[0..B) (host) in the handle's batch buffers
int search(rt_t* R, const int* origins, int B, unsigned long long* relax) {
    int rc = ensure_batch(R, B);
    if (rc) return rc;
    if ((rc = rh2d(R, R->d_origins, origins, (size_t)B))) return rc;
    return search_in(R, handle_bufs(R), B, relax);
}

int check_weight_sum(rt_t* R, unsigned long long* word) {
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(kWave), 0, R->stream, nullptr, word);
    hipLaunchKernelGGL(k_weight_sum, dim3(grid_for(R->ne)), dim3(kBlock), 0, R->stream, R->d_w, R->ne, word);
    RCHECK(R, hipGetLastError());
    unsigned long long s = 0;
    RCHECK(R, hipMemcpyAsync(&s, word, sizeof(s), hipMemcpyDeviceToHost, R->stream));
    RCHECK(R, hipStreamSynchronize(R->stream));
    if (s >= (1ull << (64 - kEdgeBits))) return rfail(R, SIM_EINVAL, "weights sum to 2^40 ms or more");
    R->wsum = (long long)s;
    return SIM_OK;
}

// Search scratch of rt_tree_static: one array per GPU, in the code object,
// so that the call allocates nothing.  Host code never uses the array's name
// as an address (it stands for a host-side shadow); every call on a device
// first looks up the device address of that device's copy.
static __device__ __align__(256) unsigned char scratch[RT_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// byte layout of the static scratch for a network of nn nodes (one origin):
// counters, relaxation word, origin, then the per-node arrays; returns the
// bytes needed
size_t static_layout(long long nn, SearchBufs* b, unsigned char* base) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return base + at;
    };
    unsigned char* cnt = take(5 * sizeof(unsigned));
    unsigned char* u64 = take(2 * sizeof(unsigned long long));
    unsigned char* org = take(sizeof(int));
    unsigned char* key = take(sizeof(unsigned long long) * nn);
    unsigned char* st = take(sizeof(unsigned) * nn);
    unsigned char* fst = take(sizeof(unsigned) * nn);
    unsigned char* f0 = take(sizeof(unsigned) * nn);
    unsigned char* f1 = take(sizeof(unsigned) * nn);
    unsigned char* r0 = take(sizeof(unsigned) * nn);
    unsigned char* r1 = take(sizeof(unsigned) * nn);
    if (b) {
        b->cnt = reinterpret_cast<unsigned*>(cnt);
        b->u64 = reinterpret_cast<unsigned long long*>(u64);
        b->origins = reinterpret_cast<int*>(org);
        b->key = reinterpret_cast<unsigned long long*>(key);
        b->stamp = reinterpret_cast<unsigned*>(st);
        b->fstamp = reinterpret_cast<unsigned*>(fst);
        b->fr[0] = reinterpret_cast<unsigned*>(f0);
        b->fr[1] = reinterpret_cast<unsigned*>(f1);
        b->far[0] = reinterpret_cast<unsigned*>(r0);
        b->far[1] = reinterpret_cast<unsigned*>(r1);
    }
    return o;
}

// device address of the current device's static scratch (looked up once per
// device); nullptr with the HIP error in *he on failure
unsigned char* static_scratch(int dev, hipError_t* he) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        *he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*he != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *he = hipSuccess;
    return g_scratch_ptr[dev];
}

__global__ void k_set_origin(int* o, int v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *o = v;
}

}  // namespace

extern "C" {

int rt_create(const sim_network* net, void* hip_stream, sim_alloc_fn alloc, sim_free_fn free_fn, void* alloc_ctx,
              rt_t** out) {
    if (!net || !out || !net->row_ptr || !net->col_idx || !net->lanes || !net->length_m || !net->speed_mps)
        return SIM_EINVAL;
    if ((alloc == nullptr) != (free_fn == nullptr)) return SIM_EINVAL;
    const int nn = net->num_nodes, ne = net->num_edges;
    if (nn <= 0 || ne <= 0 || (unsigned long long)ne >= kEdgeMask || net->row_ptr[0] != 0 ||
        net->row_ptr[nn] != ne)
        return SIM_EINVAL;
    for (int u = 0; u < nn; ++u)
        if (net->row_ptr[u + 1] < net->row_ptr[u]) return SIM_EINVAL;
    for (int e = 0; e < ne; ++e)
        if (net->col_idx[e] < 0 || net->col_idx[e] >= nn || net->lanes[e] < 1 || !(net->speed_mps[e] > 0) ||
            !(net->length_m[e] >= 0) || !std::isfinite(net->length_m[e]) || !std::isfinite(net->speed_mps[e]))
            return SIM_EINVAL;
    rt_t* R = new rt_t();
    if (hipGetDevice(&R->device) != hipSuccess) {
        (void)hipGetLastError();
        delete R;
        return SIM_EHIP;
    }
    R->stream = static_cast<hipStream_t>(hip_stream);
    R->alloc = alloc;
    R->free_fn = free_fn;
    R->ctx = alloc_ctx;
    R->nn = nn;
    R->ne = ne;
    R->row_ptr.assign(net->row_ptr, net->row_ptr + nn + 1);
    R->col_idx.assign(net->col_idx, net->col_idx + ne);
    R->lanes.assign(net->lanes, net->lanes + ne);
    R->len.assign(net->length_m, net->length_m + ne);
    R->speed.assign(net->speed_mps, net->speed_mps + ne);
    std::vector<int> tail(ne);
    for (int u = 0; u < nn; ++u)
        for (int e = R->row_ptr[u]; e < R->row_ptr[u + 1]; ++e) tail[e] = u;
    int rc = SIM_OK;
    if (!ra(R, R->d_row_ptr, nn + 1) || !ra(R, R->d_col, ne) || !ra(R, R->d_tail, ne) || !ra(R, R->d_w, ne) ||
        !ra(R, R->d_u64, 2) || !ra(R, R->d_err, 1) || !ra(R, R->d_cnt, 5))
        rc = SIM_ENOMEM;
    if (rc == SIM_OK && ((rc = rh2d(R, R->d_row_ptr, R->row_ptr.data(), nn + 1)) ||
                         (rc = rh2d(R, R->d_col, R->col_idx.data(), ne)) || (rc = rh2d(R, R->d_tail, tail.data(), ne))))
        rc = SIM_EHIP;
    if (rc == SIM_OK) rc = rt_weights_initial(R);
    if (rc == SIM_OK && hipStreamSynchronize(R->stream) != hipSuccess) rc = SIM_EHIP;
    if (rc != SIM_OK) {
        rt_destroy(R);
        return rc;
    }
    *out = R;
    return SIM_OK;
}

int rt_set_trips(rt_t* R, int32_t num_sources, const int32_t* src_nodes, int32_t num_trips, const int32_t* trip_src,
                 const int32_t* trip_dst) {
    if (!R || num_sources <= 0 || num_trips < 0 || !src_nodes || (num_trips > 0 && (!trip_src || !trip_dst)))
        return SIM_EINVAL;
    for (int s = 0; s < num_sources; ++s)
        if (src_nodes[s] < 0 || src_nodes[s] >= R->nn) return rfail(R, SIM_EINVAL, "origin node out of range");
    for (int i = 0; i < num_trips; ++i) {
        if (trip_src[i] < 0 || trip_src[i] >= num_sources || trip_dst[i] < 0 || trip_dst[i] >= R->nn)
            return rfail(R, SIM_EINVAL, "trip " + std::to_string(i) + " out of range");
        if (src_nodes[trip_src[i]] == trip_dst[i])
            return rfail(R, SIM_EINVAL, "trip " + std::to_string(i) + " ends at its origin");
    }
    for (void* p : {(void*)R->d_src_nodes, (void*)R->d_trip_src, (void*)R->d_trip_dst, (void*)R->d_pred,
                    (void*)R->d_sel, (void*)R->d_len, (void*)R->d_tsum, (void*)R->d_ptr, (void*)R->d_edges})
        rfree(R, p);
    R->d_src_nodes = R->d_trip_src = R->d_trip_dst = R->d_pred = R->d_edges = nullptr;
    R->d_sel = nullptr;
    R->d_len = R->d_tsum = R->d_ptr = nullptr;
    R->have_routes = false;
    R->total = 0;
    R->nsrc = num_sources;
    R->ntrips = num_trips;
    R->h_src_nodes.assign(src_nodes, src_nodes + num_sources);
    R->h_trip_src.assign(trip_src, trip_src + num_trips);
    const size_t n = (size_t)num_trips;
    const int ntiles = (int)((n + kScanTile - 1) / kScanTile);
    if (!ra(R, R->d_src_nodes, num_sources) || !ra(R, R->d_trip_src, n) || !ra(R, R->d_trip_dst, n) ||
        !ra(R, R->d_pred, (size_t)num_sources * (size_t)R->nn) || !ra(R, R->d_sel, n) || !ra(R, R->d_len, n) ||
        !ra(R, R->d_tsum, (size_t)std::max(ntiles, 1)))
        return rfail(R, SIM_ENOMEM, "trip arrays (including one predecessor array per origin) do not fit");
    int rc;
    if ((rc = rh2d(R, R->d_src_nodes, src_nodes, (size_t)num_sources)) || (rc = rh2d(R, R->d_trip_src, trip_src, n)) ||
        (rc = rh2d(R, R->d_trip_dst, trip_dst, n)))
        return rc;
    RCHECK(R, hipStreamSynchronize(R->stream));
    return SIM_OK;
}

int rt_weights_initial(rt_t* R) {
    if (!R) return SIM_EINVAL;
    std::vector<long long> w(R->ne);
    for (int e = 0; e < R->ne; ++e) {
        const double ms = std::sqrt((double)R->lanes[e]) * (double)R->len[e] / (double)R->speed[e] * 1000.0;
        const double r = std::floor(ms + 0.5);
        w[e] = r < 1.0 ? 1 : (long long)r;
    }
    int rc = rh2d(R, R->d_w, w.data(), (size_t)R->ne);
    if (rc) return rc;
    RCHECK(R, hipStreamSynchronize(R->stream));
    return SIM_OK;
}

int rt_weights_from_stats(rt_t* R, const int64_t* edge_count, const int64_t* edge_tt_us) {
    if (!R || !edge_count || !edge_tt_us) return SIM_EINVAL;
    hipLaunchKernelGGL(k_weights_from_stats, dim3(grid_for(R->ne)), dim3(kBlock), 0, R->stream,
                       (const long long*)edge_count, (const long long*)edge_tt_us, R->d_w, R->ne);
    RCHECK(R, hipGetLastError());
    return SIM_OK;
}

int rt_set_weights(rt_t* R, const int64_t* weights_ms) {
    if (!R || !weights_ms) return SIM_EINVAL;
    for (int e = 0; e < R->ne; ++e)
        if (weights_ms[e] < 1) return rfail(R, SIM_EINVAL, "weight of edge " + std::to_string(e) + " < 1");
    int rc = rh2d(R, R->d_w, (const long long*)weights_ms, (size_t)R->ne);
    if (rc) return rc;
    RCHECK(R, hipStreamSynchronize(R->stream));
    return SIM_OK;
}

int rt_read_weights(rt_t* R, int64_t* weights_ms) {
    if (!R || !weights_ms) return SIM_EINVAL;
    RCHECK(R, hipMemcpyAsync(weights_ms, R->d_w, sizeof(long long) * R->ne, hipMemcpyDeviceToHost, R->stream));
    RCHECK(R, hipStreamSynchronize(R->stream));
    return SIM_OK;
}

int rt_plan(rt_t* R, const uint8_t* select, int64_t* total_route_edges) {
    if (!R || !total_route_edges) return SIM_EINVAL;
    if (R->nsrc == 0) return rfail(R, SIM_ESTATE, "no trips set");
    if (select && !R->have_routes) return rfail(R, SIM_ESTATE, "a partial plan needs current routes");
    int rc = check_weight_sum(R, R->d_u64 + 1);
    if (rc) return rc;
    const int n = R->ntrips;
    // origins with a selected trip
    std::vector<unsigned char> need(R->nsrc, 0);
    for (int i = 0; i < n; ++i)
        if (!select || select[i]) need[R->h_trip_src[i]] = 1;
    std::vector<int> todo;  // origin indices
    for (int s = 0; s < R->nsrc; ++s)
        if (need[s]) todo.push_back(s);
    // automatic: at least the batch the router already holds memory for (its
    // own buffers no longer count as free)
    const int B = R->batch > 0 ? R->batch : std::max(auto_batch(R), R->batch_alloc);
    unsigned long long relax = 0;
    std::vector<int> nodes;
    for (size_t b0 = 0; b0 < todo.size(); b0 += (size_t)B) {
        const int nb = (int)std::min<size_t>((size_t)B, todo.size() - b0);
        nodes.resize(nb);
        for (int k = 0; k < nb; ++k) nodes[k] = R->h_src_nodes[todo[b0 + k]];
        if ((rc = search(R, nodes.data(), nb, &relax))) return rc;
        // predecessor arrays: origins of a batch are consecutive in todo but
        // not in the per-origin array, so extract one origin at a time
        for (int k = 0; k < nb; ++k)
            hipLaunchKernelGGL(k_preds, dim3(grid_for(R->nn)), dim3(kBlock), 0, R->stream,
                               R->d_key + (size_t)k * R->nn, (long long)R->nn,
                               R->d_pred + (size_t)todo[b0 + k] * R->nn);
        RCHECK(R, hipGetLastError());
    }
    R->last_relax = (long long)relax;
    R->last_sources = (int)todo.size();
    if (select && (rc = rh2d(R, R->d_sel, select, (size_t)n))) return rc;
    TripView T{R->d_trip_src, R->d_trip_dst, R->d_src_nodes, R->d_pred, R->d_tail, (long long)R->nn, n,
               select ? R->d_sel : nullptr};
    long long* nptr = nullptr;
    if (!ra(R, nptr, (size_t)n + 1)) return rfail(R, SIM_ENOMEM, "route pointer array");
    RCHECK(R, hipMemsetAsync(R->d_err, 0, sizeof(unsigned), R->stream));
    hipLaunchKernelGGL(k_route_len, dim3(grid_for(n)), dim3(kBlock), 0, R->stream, T, R->d_ptr, R->d_len, R->d_err);
    const int ntiles = (n + kScanTile - 1) / kScanTile;
    if (n > 0) {
        hipLaunchKernelGGL(k_tile_sums, dim3(ntiles), dim3(kBlock), 0, R->stream, R->d_len, n, R->d_tsum);
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, R->stream, R->d_tsum, ntiles);
        hipLaunchKernelGGL(k_tile_apply, dim3(ntiles), dim3(kBlock), 0, R->stream, R->d_len, n, R->d_tsum, nptr);
    } else {
        RCHECK(R, hipMemsetAsync(nptr, 0, sizeof(long long), R->stream));
    }
    RCHECK(R, hipGetLastError());
    unsigned e = 0;
    long long total = 0;
    RCHECK(R, hipMemcpyAsync(&e, R->d_err, sizeof(e), hipMemcpyDeviceToHost, R->stream));
    RCHECK(R, hipMemcpyAsync(&total, nptr + n, sizeof(total), hipMemcpyDeviceToHost, R->stream));
    RCHECK(R, hipStreamSynchronize(R->stream));
    if (e) {
        rfree(R, nptr);
        return rfail(R, SIM_EROUTE, "a selected destination is unreachable from its origin");
    }
    int* nedges = nullptr;
    if (!ra(R, nedges, (size_t)std::max<long long>(total, 1))) {
        rfree(R, nptr);
        return rfail(R, SIM_ENOMEM, "route array of " + std::to_string(total) + " edges");
    }
    hipLaunchKernelGGL(k_route_write, dim3(grid_for(n)), dim3(kBlock), 0, R->stream, T, R->d_ptr, R->d_edges, nptr,
                       nedges);
    RCHECK(R, hipGetLastError());
    RCHECK(R, hipStreamSynchronize(R->stream));
    rfree(R, R->d_ptr);
    rfree(R, R->d_edges);
    R->d_ptr = nptr;
    R->d_edges = nedges;
    R->total = total;
    R->have_routes = true;
    *total_route_edges = total;
    return SIM_OK;
}

int rt_read_routes(rt_t* R, int64_t* route_ptr, int32_t* route_edges) {
    if (!R) return SIM_EINVAL;
    if (!R->have_routes) return rfail(R, SIM_ESTATE, "no routes planned");
    if (route_ptr)
        RCHECK(R, hipMemcpyAsync(route_ptr, R->d_ptr, sizeof(long long) * ((size_t)R->ntrips + 1),
                                 hipMemcpyDeviceToHost, R->stream));
    if (route_edges && R->total > 0)
        RCHECK(R, hipMemcpyAsync(route_edges, R->d_edges, sizeof(int) * (size_t)R->total, hipMemcpyDeviceToHost,
                                 R->stream));
    RCHECK(R, hipStreamSynchronize(R->stream));
    return SIM_OK;
}

int rt_route_views(rt_t* R, const int64_t** route_ptr, const int32_t** route_edges, int64_t* total_route_edges) {
    if (!R) return SIM_EINVAL;
    if (!R->have_routes) return rfail(R, SIM_ESTATE, "no routes planned");
    if (route_ptr) *route_ptr = reinterpret_cast<const int64_t*>(R->d_ptr);
    if (route_edges) *route_edges = R->d_edges;
    if (total_route_edges) *total_route_edges = R->total;
    return SIM_OK;
}

int rt_tree(rt_t* R, int32_t src_node, int64_t* dist, int32_t* pred) {
    if (!R || src_node < 0 || src_node >= R->nn) return SIM_EINVAL;
    int rc = check_weight_sum(R, R->d_u64 + 1);
    if (rc) return rc;
    unsigned long long relax = 0;
    if ((rc = search(R, &src_node, 1, &relax))) return rc;
    long long* dd = nullptr;
    int* pp = nullptr;
    if (!ra(R, dd, (size_t)R->nn) || !ra(R, pp, (size_t)R->nn)) {
        rfree(R, dd);
        rfree(R, pp);
        return rfail(R, SIM_ENOMEM, "tree arrays");
    }
    hipLaunchKernelGGL(k_dists, dim3(grid_for(R->nn)), dim3(kBlock), 0, R->stream, R->d_key, (long long)R->nn, dd);
    hipLaunchKernelGGL(k_preds, dim3(grid_for(R->nn)), dim3(kBlock), 0, R->stream, R->d_key, (long long)R->nn, pp);
    hipError_t he = hipGetLastError();
    if (he == hipSuccess && dist)
        he = hipMemcpyAsync(dist, dd, sizeof(long long) * R->nn, hipMemcpyDeviceToHost, R->stream);
    if (he == hipSuccess && pred) he = hipMemcpyAsync(pred, pp, sizeof(int) * R->nn, hipMemcpyDeviceToHost, R->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(R->stream);
    rfree(R, dd);
    rfree(R, pp);
    if (he != hipSuccess) {
        (void)hipGetLastError();
        return rfail(R, SIM_EHIP, std::string("rt_tree: ") + hipGetErrorString(he));
    }
    return SIM_OK;
}

int rt_tree_static(rt_t* R, int32_t src_node, int64_t* dist, int32_t* pred) {
    if (!R || src_node < 0 || src_node >= R->nn) return SIM_EINVAL;
    const size_t need = static_layout(R->nn, nullptr, nullptr);
    if (need > (size_t)RT_STATIC_SCRATCH_BYTES)
        return rfail(R, SIM_EINVAL, "rt_tree_static: a network of " + std::to_string(R->nn) + " nodes needs " +
                                        std::to_string(need) + " bytes of search scratch, the static buffer holds " +
                                        std::to_string((size_t)RT_STATIC_SCRATCH_BYTES));
    int dev = -1;
    RCHECK(R, hipGetDevice(&dev));
    if (dev != R->device || dev < 0 || dev >= kMaxDevices)
        return rfail(R, SIM_EINVAL, "rt_tree_static: call it with the router's device current");
    hipError_t he = hipSuccess;
    unsigned char* base = static_scratch(dev, &he);
    if (!base) return rfail(R, SIM_EHIP, std::string("rt_tree_static: hipGetSymbolAddress: ") + hipGetErrorString(he));
    SearchBufs b{};
    static_layout(R->nn, &b, base);
    int rc = check_weight_sum(R, b.u64 + 1);
    if (rc) return rc;
    hipLaunchKernelGGL(k_set_origin, dim3(1), dim3(kWave), 0, R->stream, b.origins, (int)src_node);
    unsigned long long relax = 0;
    if ((rc = search_in(R, b, 1, &relax))) return rc;
    if (dist)
        hipLaunchKernelGGL(k_dists, dim3(grid_for(R->nn)), dim3(kBlock), 0, R->stream, b.key, (long long)R->nn,
                           (long long*)dist);
    if (pred)
        hipLaunchKernelGGL(k_preds, dim3(grid_for(R->nn)), dim3(kBlock), 0, R->stream, b.key, (long long)R->nn,
                           (int*)pred);
    RCHECK(R, hipGetLastError());
    RCHECK(R, hipStreamSynchronize(R->stream));
    return SIM_OK;
}

int rt_last_work(rt_t* R, int64_t* relaxations, int32_t* sources) {
    if (!R) return SIM_EINVAL;
    if (relaxations) *relaxations = R->last_relax;
    if (sources) *sources = R->last_sources;
    return SIM_OK;
}

int rt_set_batch(rt_t* R, int32_t sources_per_batch) {
    if (!R || sources_per_batch < 0) return SIM_EINVAL;
    if (sources_per_batch > 0 && (unsigned long long)sources_per_batch * (unsigned long long)R->nn > UINT32_MAX)
        return rfail(R, SIM_EINVAL, "batch x nodes must stay below 2^32");
    R->batch = sources_per_batch;
    return SIM_OK;
}

int rt_set_delta(rt_t* R, int64_t delta_ms) {
    if (!R || delta_ms < 0) return SIM_EINVAL;
    R->delta = delta_ms;
    return SIM_OK;
}

int rt_set_stream(rt_t* R, void* hip_stream) {
    if (!R) return SIM_EINVAL;
    RCHECK(R, hipStreamSynchronize(R->stream));
    R->stream = static_cast<hipStream_t>(hip_stream);
    return SIM_OK;
}

const char* rt_last_error(const rt_t* R) { return R ? R->err.c_str() : "null handle"; }

void rt_destroy(rt_t* R) {
    if (!R) return;
    (void)hipStreamSynchronize(R->stream);
    for (void* p : R->allocs) {
        if (R->free_fn) R->free_fn(R->ctx, p);
        else (void)hipFree(p);
    }
    R->allocs.clear();
    delete R;
}

}  // extern "C"
