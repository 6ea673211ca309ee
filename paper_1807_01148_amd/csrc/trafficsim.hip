// libtrafficsim: the traffic microsimulation step of Waddell et al., Sec. 6,
// as hand-written HIP for CDNA4 (gfx950).
//
// One synchronous step t -> t+1 (every decision reads state t only):
//   k_decide   per vehicle: leader search, IDM acceleration (Sec. 6.3.2,
//              car-following equation), ballistic update, link-end crossing or
//              arrival (Sec. 6.3.1 routes), lane-change intent with gap
//              acceptance (Sec. 6.3.2 lane changing / gap acceptance);
//              per due trip (Sec. 6.2.2): entry-lane choice.  Crossings, lane
//              changes and insertions claim one-metre cells of their target
//              lane with a 64-bit atomicMin of (epoch, vehicle id).
//   k_resolve  per claim: it wins iff it still owns all its cells (no
//              overlapping claim with a lower id); winners locate their gap in
//              the sorted order by binary search and take a slot in it.
//   k_scan     exclusive scan (decoupled look-back) of stay[i] + movers-in-gap[i]
//              gives every survivor and every mover its new position.
//   k_scatter  survivors write their record to the new buffer; movers stage
//              their (lane, x) keys per gap.
//   k_place    movers rank themselves inside their gap and write their
//              record; the last block advances the device-side counters.
//
// Vehicle state is structure-of-arrays, double-buffered, kept sorted by
// (global lane id, position), so the vehicle ahead in the lane is the next
// array element (coalesced) and the lane of another link is found by binary
// search over the sorted keys.  The whole loop runs without host round trips.
//
// Floating point: built with -ffp-contract=off; every expression below is
// evaluated in float in the order written (correctly rounded divide), so a
// CPU float implementation of the same rules reproduces it bit for bit.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "trafficsim.h"

namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kLcNone = -(1 << 30);
constexpr int kMaxGrid = 2048;

enum : int { kCross = 1, kChange = 2, kInsert = 3 };

// ---------------------------------------------------------------------------
// device-side data
// ---------------------------------------------------------------------------
struct Counters {
    int t;           // current step
    int n;           // vehicles on the road (entries of the current buffer)
    int npend;       // carried insertion candidates (current pending buffer)
    int nclaim;      // claims this step
    int nmove;       // winning claims this step
    int npend_next;  // candidates carried to the next step
    int n_next;      // entries of the next buffer
    unsigned scan_tile;
    unsigned done_blocks;
    int pad;
    unsigned long long arrived, departed, updates, claims_lost, clamps, claims;
};

struct Params {
    float dt, h, lveh, s0, claim_len, s_eps, b_max, pol, athr, bsafe, dmand, dt_us_f;
    long long dt_us;
    int lc_cool;
};

struct Net {
    const float* len;
    const float* inv_v0;
    const int* lane_base;
    const int* lanes;
    const int* cls;
    const int* head;
    const int* row_ptr;
    const long long* cbase;  // first claim cell of lane 0 of the edge
    const int* ncell;        // cells per lane = floor(len) + 1
    const float* cT;
    const float* cA;
    const float* cKab;
};

struct Trips {
    const int* route_edges;
    const int* rbeg;
    const int* rend;
    const int* rel_off;  // rel_off[t] = first vehicle id due at step >= t
    int rel_len;         // rel_off has rel_len + 1 entries
    const unsigned char* placed;
    int* depart_actual;
    int* arrive_step;
};

struct Veh {
    int* key;
    float* x;
    float* v;
    int* edge;
    int* rcur;
    int* next;
    int* lc;
    int* kin;
    float* phin;
    int* vid;
};

struct Scratch {
    float* xs;
    float* vs;
    unsigned char* stay;
    int* mcnt;
    int* cscan;
    int* cl_vid;
    int* cl_key;
    int* cl_lo;
    int* cl_hi;
    int* cl_src;
    int* cl_kind;
    int* cl_tedge;
    float* cl_X;
    float* cl_v;
    float* cl_f;
    int* mv_claim;
    int* mv_p;
    int* mv_slot;
    int* mv_g;
    int* grp_key;
    float* grp_X;
    unsigned long long* cells;
    unsigned long long* tile_status;
    unsigned long long* st_cnt;
    unsigned long long* st_steps;
    unsigned long long* st_us;
};

struct Lead {
    int kind;  // 0 free road, 1 same link, 2 rearmost vehicle of the next link
    float s;   // bumper-to-bumper gap
    float vl;  // speed of the vehicle ahead
    float xl;  // its position on its own link
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fmx(float a, float b) { return a > b ? a : b; }
__device__ __forceinline__ float fmn(float a, float b) { return a < b ? a : b; }

// IDM (Sec. 6.3.2, car-following equation, exponent 4): dynamic part of the
// desired gap floored at 0, gap floored at s_eps, result floored at -b_max.
__device__ __forceinline__ float idm_acc(const Params& P, float A, float T, float kab, float iv,
                                         float v, const Lead& L) {
    float r = v * iv;
    float r2 = r * r;
    float r4 = r2 * r2;
    float fr = 1.0f - r4;
    float acc;
    if (L.kind == 0) {
        acc = A * fr;
    } else {
        float dv = v - L.vl;
        float dyn = v * T + (v * dv) * kab;
        float ss = P.s0 + fmx(0.0f, dyn);
        float q = ss / fmx(L.s, P.s_eps);
        acc = A * (fr - q * q);
    }
    return fmx(acc, -P.b_max);
}

// ballistic update; stop inside the step when the speed would turn negative
__device__ __forceinline__ void kin_move(const Params& P, float v, float acc, float& dx, float& vn) {
    float vv = v + acc * P.dt;
    if (vv < 0.0f) {
        dx = (v * v) / (-2.0f * acc);
        vn = 0.0f;
    } else {
        dx = v * P.dt + acc * P.h;
        vn = vv;
    }
    dx = fmx(dx, 0.0f);
}

__device__ __forceinline__ int clamp_to_leader(const Lead& L, float& dx, float& vn) {
    if (L.kind != 0 && dx > L.s) {
        dx = fmx(L.s, 0.0f);
        vn = fmn(vn, L.vl);
        return 1;
    }
    return 0;
}

__device__ __forceinline__ Lead relead(const Params& P, float len, const Lead& L, float xf) {
    Lead R = L;
    if (L.kind == 1) R.s = (L.xl - P.lveh) - xf;
    else if (L.kind == 2) R.s = (len - xf) + (L.xl - P.lveh);
    return R;
}

// first j in [lo, hi) with key[j] >= k
__device__ __forceinline__ int lb_key(const int* __restrict__ key, int lo, int hi, int k) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (key[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first j in [lo, hi) with (key[j], x[j]) >= (k, X)
__device__ __forceinline__ int lb_keyx(const int* __restrict__ key, const float* __restrict__ x, int lo,
                                       int hi, int k, float X) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int km = key[mid];
        if (km < k || (km == k && x[mid] < X)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first j in [lo, hi) with (key[j], x[j]) > (k, X)
__device__ __forceinline__ int ub_keyx(const int* __restrict__ key, const float* __restrict__ x, int lo,
                                       int hi, int k, float X) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int km = key[mid];
        if (km < k || (km == k && x[mid] <= X)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long epoch_tag(int t) {
    return (unsigned long long)(0xFFFFFFFFu - (unsigned)t) << 32;
}

__device__ __forceinline__ void claim_cells(const Params& P, const Net& net, int edge, float X, int& lo,
                                            int& hi) {
    int a = (int)floorf(X - P.claim_len);
    int b = (int)floorf(X);
    int nc = net.ncell[edge];
    lo = a < 0 ? 0 : a;
    hi = b > nc - 1 ? nc - 1 : b;
}

__device__ __forceinline__ void push_claim(const Scratch& s, const Net& net, Counters* ctr,
                                           unsigned long long tag, int vid, int kind, int src,
                                           int tedge, int tlane, float X, float vc, float f, int lo,
                                           int hi) {
    int ci = atomicAdd(&ctr->nclaim, 1);
    s.cl_vid[ci] = vid;
    s.cl_key[ci] = net.lane_base[tedge] + tlane;
    s.cl_lo[ci] = lo;
    s.cl_hi[ci] = hi;
    s.cl_src[ci] = src;
    s.cl_kind[ci] = kind;
    s.cl_tedge[ci] = tedge;
    s.cl_X[ci] = X;
    s.cl_v[ci] = vc;
    s.cl_f[ci] = f;
    unsigned long long* cell = s.cells + net.cbase[tedge] + (long long)tlane * net.ncell[tedge];
    unsigned long long mine = tag | (unsigned)vid;
    for (int c = lo; c <= hi; ++c) atomicMin(cell + c, mine);
}

__device__ __forceinline__ void record_exit(const Params& P, const Scratch& s, int edge, int kin,
                                            float phin, float f, int t) {
    long long ns = (long long)(t + 1) - kin;
    float frac = f - phin;
    long long us = ns * P.dt_us + (long long)rintf(frac * P.dt_us_f);
    atomicAdd(s.st_cnt + edge, 1ull);
    atomicAdd(s.st_steps + edge, (unsigned long long)ns);
    atomicAdd(s.st_us + edge, (unsigned long long)us);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// k_decide
// ---------------------------------------------------------------------------
__device__ void decide_vehicle(const Params& P, const Net& net, const Trips& tr, const Veh& in,
                               const Scratch& s, Counters* ctr, int N, int t,
                               unsigned long long tag, int i, int& clamps, int& arrivals) {
    const int k = in.key[i];
    const float x = in.x[i];
    const float v = in.v[i];
    const int e = in.edge[i];
    const int nx = in.next[i];
    const float len = net.len[e];
    const float iv = net.inv_v0[e];
    const int c = net.cls[e];
    const float A = net.cA[c], T = net.cT[c], kab = net.cKab[c];
    const int lb = net.lane_base[e];
    const int l = k - lb;

    // own leader: next element of the lane, else the rearmost vehicle of the
    // mapped lane of the next link of the route
    Lead L = {0, 0.0f, 0.0f, 0.0f};
    if (i + 1 < N && in.key[i + 1] == k) {
        float xl = in.x[i + 1];
        L.kind = 1; L.xl = xl; L.vl = in.v[i + 1]; L.s = (xl - P.lveh) - x;
    } else if (nx >= 0) {
        int nl2 = net.lanes[nx];
        int k2 = net.lane_base[nx] + (l < nl2 - 1 ? l : nl2 - 1);
        int j = lb_key(in.key, 0, N, k2);
        if (j < N && in.key[j] == k2) {
            float xl = in.x[j];
            L.kind = 2; L.xl = xl; L.vl = in.v[j]; L.s = (len - x) + (xl - P.lveh);
        }
    }
    const float ac = idm_acc(P, A, T, kab, iv, v, L);
    float dx, vn;
    kin_move(P, v, ac, dx, vn);
    clamps += clamp_to_leader(L, dx, vn);
    const float xs = x + dx;
    const int vid = in.vid[i];

    if (xs > len) {  // the front passes the link end strictly
        float f = dx > 0.0f ? fmn((len - x) / dx, 1.0f) : 0.0f;
        if (nx < 0) {  // arrival at the end of the last link
            record_exit(P, s, e, in.kin[i], in.phin[i], f, t);
            tr.arrive_step[vid] = t + 1;
            s.stay[i] = 0;
            arrivals += 1;
            return;
        }
        int nl2 = net.lanes[nx];
        int tl = l < nl2 - 1 ? l : nl2 - 1;
        float X = xs - len;
        int lo, hi;
        claim_cells(P, net, nx, X, lo, hi);
        s.xs[i] = len;  // outcome if the claim is lost: wait at the link end
        s.vs[i] = 0.0f;
        s.stay[i] = 1;
        push_claim(s, net, ctr, tag, vid, kCross, i, nx, tl, X, vn, f, lo, hi);
        return;
    }
    s.xs[i] = xs;
    s.vs[i] = vn;
    s.stay[i] = 1;

    // lane change: eligibility
    const int n = net.lanes[e];
    if (n < 2 || (t - in.lc[i]) < P.lc_cool || x < P.lveh) return;
    int blo = 0, bhi = n - 1;
    if (nx >= 0) {
        int hn = net.head[e];
        int r0 = net.row_ptr[hn];
        int m = net.row_ptr[hn + 1] - r0;
        int j = nx - r0;
        blo = (j * n) / m;
        bhi = ((j + 1) * n + m - 1) / m - 1;
        if (bhi < blo) bhi = blo;
    }
    const float d = len - x;
    const bool inband = blo <= l && l <= bhi;
    const bool mand = !inband && d <= P.dmand;
    int cand[2];
    int nc = 0;
    if (mand) {
        cand[nc++] = l < blo ? l + 1 : l - 1;
    } else {
        for (int sd = l - 1; sd <= l + 1; sd += 2) {
            if (sd < 0 || sd >= n) continue;
            if (inband && d <= P.dmand && (sd < blo || sd > bhi)) continue;
            cand[nc++] = sd;
        }
    }
    const bool hasF = i > 0 && in.key[i - 1] == k;
    const float xF = hasF ? in.x[i - 1] : 0.0f;
    const float vF = hasF ? in.v[i - 1] : 0.0f;

    int best = -1;
    float best_inc = 0.0f, best_X = 0.0f, best_v = 0.0f;
    for (int ci = 0; ci < nc; ++ci) {
        const int lt = cand[ci];
        const int kt = lb + lt;
        // first vehicle of the target lane strictly ahead; the one before it
        // (position <= x) is the lag
        int j = lt > l ? ub_keyx(in.key, in.x, i + 1, N, kt, x) : ub_keyx(in.key, in.x, 0, i, kt, x);
        Lead Lt = {0, 0.0f, 0.0f, 0.0f};
        if (j < N && in.key[j] == kt) {
            float xl = in.x[j];
            Lt.kind = 1; Lt.xl = xl; Lt.vl = in.v[j]; Lt.s = (xl - P.lveh) - x;
        } else if (nx >= 0) {
            int nl2 = net.lanes[nx];
            int k2 = net.lane_base[nx] + (lt < nl2 - 1 ? lt : nl2 - 1);
            int j2 = lb_key(in.key, 0, N, k2);
            if (j2 < N && in.key[j2] == k2) {
                float xl = in.x[j2];
                Lt.kind = 2; Lt.xl = xl; Lt.vl = in.v[j2]; Lt.s = (len - x) + (xl - P.lveh);
            }
        }
        const bool hasFt = j > 0 && in.key[j - 1] == kt;
        const float xFt = hasFt ? in.x[j - 1] : 0.0f;
        const float vFt = hasFt ? in.v[j - 1] : 0.0f;
        // gap acceptance (Sec. 6.3.2)
        if (Lt.kind != 0 && Lt.s < P.s0) continue;
        if (hasFt && ((x - P.lveh) - xFt) < P.s0) continue;
        const float at = idm_acc(P, A, T, kab, iv, v, Lt);
        if (at < -P.bsafe) continue;
        float dxt, vt;
        kin_move(P, v, at, dxt, vt);
        clamp_to_leader(Lt, dxt, vt);
        const float Xt = x + dxt;
        if (Xt >= len) continue;
        float an = 0.0f, ant = 0.0f;
        if (hasFt) {
            an = idm_acc(P, A, T, kab, iv, vFt, relead(P, len, Lt, xFt));
            Lead Li = {1, (x - P.lveh) - xFt, v, x};
            ant = idm_acc(P, A, T, kab, iv, vFt, Li);
            if (ant < -P.bsafe) continue;
            Lead none = {0, 0.0f, 0.0f, 0.0f};
            float afree = idm_acc(P, A, T, kab, iv, vFt, none);
            float dxF, vF2;
            kin_move(P, vFt, afree, dxF, vF2);
            if (((Xt - P.lveh) - xFt) < dxF) continue;
        }
        float inc = 0.0f;
        if (!mand) {
            float d1 = at - ac;
            float d2 = hasFt ? (ant - an) : 0.0f;
            float d3 = 0.0f;
            if (hasF) {
                Lead Lo = {1, (x - P.lveh) - xF, v, x};
                float ao = idm_acc(P, A, T, kab, iv, vF, Lo);
                float aot = idm_acc(P, A, T, kab, iv, vF, relead(P, len, L, xF));
                d3 = aot - ao;
            }
            inc = d1 + P.pol * (d2 + d3);
            if (!(inc > P.athr)) continue;
        }
        if (best < 0 || inc > best_inc) {
            best = lt; best_inc = inc; best_X = Xt; best_v = vt;
        }
    }
    if (best >= 0) {
        int lo, hi;
        claim_cells(P, net, e, best_X, lo, hi);
        push_claim(s, net, ctr, tag, vid, kChange, i, e, best, best_X, best_v, 0.0f, lo, hi);
    }
}

__device__ void decide_insert(const Params& P, const Net& net, const Trips& tr, const Veh& in,
                              const Scratch& s, Counters* ctr, int* pend_out, int N,
                              unsigned long long tag, int vid) {
    if (tr.placed[vid]) return;
    const int e0 = tr.route_edges[tr.rbeg[vid]];
    const int n0 = net.lanes[e0];
    const int lb = net.lane_base[e0];
    const float len0 = net.len[e0];
    int j = lb_key(in.key, 0, N, lb);
    int best = -1;
    float bsp = 0.0f;
    for (int l = 0; l < n0; ++l) {
        const int kk = lb + l;
        while (j < N && in.key[j] < kk) ++j;
        float sp = (j < N && in.key[j] == kk) ? (in.x[j] - P.lveh) : len0;
        if (best < 0 || sp > bsp) { best = l; bsp = sp; }
    }
    if (bsp >= P.claim_len) {
        int lo, hi;
        claim_cells(P, net, e0, P.lveh, lo, hi);
        push_claim(s, net, ctr, tag, vid, kInsert, -1, e0, best, P.lveh, 0.0f, 1.0f, lo, hi);
    } else {
        pend_out[atomicAdd(&ctr->npend_next, 1)] = vid;
    }
}

__global__ __launch_bounds__(kBlock) void k_decide(Params P, Net net, Trips tr, Veh in, Scratch s,
                                                   const int* __restrict__ pend_in, int* pend_out,
                                                   Counters* ctr) {
    const int t = ctr->t;
    const int N = ctr->n;
    const int np = ctr->npend;
    int rlo = 0, rhi = 0;
    if (t < tr.rel_len) {
        rlo = tr.rel_off[t];
        rhi = tr.rel_off[t + 1];
    }
    const int total = N + np + (rhi - rlo);
    const unsigned long long tag = epoch_tag(t);
    int clamps = 0, arrivals = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
        if (i < N) {
            decide_vehicle(P, net, tr, in, s, ctr, N, t, tag, i, clamps, arrivals);
        } else {
            int cidx = i - N;
            int vid = cidx < np ? pend_in[cidx] : rlo + (cidx - np);
            decide_insert(P, net, tr, in, s, ctr, pend_out, N, tag, vid);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) s.stay[N] = 0;
    unsigned long long cw = wave_sum_u64((unsigned long long)clamps);
    unsigned long long aw = wave_sum_u64((unsigned long long)arrivals);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (cw) atomicAdd(&ctr->clamps, cw);
        if (aw) atomicAdd(&ctr->arrived, aw);
    }
}

// ---------------------------------------------------------------------------
// k_resolve
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_resolve(Params P, Net net, Trips tr, Veh in, Scratch s,
                                                    int* pend_out, Counters* ctr) {
    const int t = ctr->t;
    const int N = ctr->n;
    const int C = ctr->nclaim;
    const unsigned long long tag = epoch_tag(t);
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->scan_tile = 0;
    int lost = 0, departed = 0;
    for (int ci = blockIdx.x * kBlock + threadIdx.x; ci < C; ci += gridDim.x * kBlock) {
        const int vid = s.cl_vid[ci];
        const int tedge = s.cl_tedge[ci];
        const int key = s.cl_key[ci];
        const int tl = key - net.lane_base[tedge];
        const unsigned long long* cell = s.cells + net.cbase[tedge] + (long long)tl * net.ncell[tedge];
        const unsigned long long mine = tag | (unsigned)vid;
        bool win = true;
        for (int c = s.cl_lo[ci]; c <= s.cl_hi[ci]; ++c) {
            if (cell[c] != mine) { win = false; break; }
        }
        const int kind = s.cl_kind[ci];
        const int src = s.cl_src[ci];
        if (win) {
            if (src >= 0) s.stay[src] = 0;
            int m = atomicAdd(&ctr->nmove, 1);
            s.mv_claim[m] = ci;
            int p = lb_keyx(in.key, in.x, 0, N, key, s.cl_X[ci]);
            s.mv_p[m] = p;
            s.mv_slot[m] = atomicAdd(&s.mcnt[p], 1);
            if (kind == kCross) record_exit(P, s, in.edge[src], in.kin[src], in.phin[src], s.cl_f[ci], t);
            if (kind == kInsert) {
                tr.depart_actual[vid] = t + 1;
                departed += 1;
            }
        } else {
            lost += 1;
            if (kind == kInsert) pend_out[atomicAdd(&ctr->npend_next, 1)] = vid;
        }
    }
    unsigned long long lw = wave_sum_u64((unsigned long long)lost);
    unsigned long long dw = wave_sum_u64((unsigned long long)departed);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (lw) atomicAdd(&ctr->claims_lost, lw);
        if (dw) atomicAdd(&ctr->departed, dw);
    }
}

// ---------------------------------------------------------------------------
// k_scan: exclusive scan of w[i] = stay[i] + mcnt[i], i in [0, N], single pass
// with decoupled look-back; tiles are handed out in order by an atomic counter
// so a tile only ever waits on tiles already being processed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int block_excl_scan(int v, int& total) {
    __shared__ int ws[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    int inc = v;
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) ws[w] = inc;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int q = 0; q < kBlock / kWave; ++q) {
        if (q < w) pre += ws[q];
        tot += ws[q];
    }
    __syncthreads();
    total = tot;
    return pre + inc - v;
}

constexpr unsigned long long kFlagA = 1ull, kFlagP = 2ull;

__device__ __forceinline__ unsigned long long pack_status(unsigned ep, unsigned long long flag, int val) {
    return ((unsigned long long)ep << 34) | (flag << 32) | (unsigned)val;
}

__global__ __launch_bounds__(kBlock) void k_scan(Scratch s, Counters* ctr) {
    const int N = ctr->n;
    const int total = N + 1;
    const int ntiles = (total + kScanTile - 1) / kScanTile;
    const unsigned ep = ((unsigned)ctr->t & 0x3FFFFFFFu) + 1u;
    __shared__ int s_tile;
    __shared__ int s_prefix;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(&ctr->scan_tile, 1u);
        __syncthreads();
        const int tile = s_tile;
        __syncthreads();
        if (tile >= ntiles) break;
        const int base = tile * kScanTile + threadIdx.x * kScanItems;
        int vals[kScanItems];
        int tsum = 0;
        for (int q = 0; q < kScanItems; ++q) {
            int idx = base + q;
            int w = 0;
            if (idx < total) w = s.mcnt[idx] + (idx < N ? (int)s.stay[idx] : 0);
            vals[q] = w;
            tsum += w;
        }
        int agg;
        int excl = block_excl_scan(tsum, agg);
        if (threadIdx.x == 0) {
            int prefix = 0;
            if (tile == 0) {
                __hip_atomic_store(&s.tile_status[0], pack_status(ep, kFlagP, agg), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __hip_atomic_store(&s.tile_status[tile], pack_status(ep, kFlagA, agg), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                int j = tile - 1;
                for (;;) {
                    unsigned long long st = __hip_atomic_load(&s.tile_status[j], __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                    unsigned sep = (unsigned)(st >> 34);
                    unsigned long long flag = (st >> 32) & 3ull;
                    if (sep != ep || flag == 0ull) {
                        __builtin_amdgcn_s_sleep(1);
                        continue;
                    }
                    prefix += (int)(unsigned)(st & 0xFFFFFFFFull);
                    if (flag == kFlagP) break;
                    --j;
                }
                __hip_atomic_store(&s.tile_status[tile], pack_status(ep, kFlagP, prefix + agg),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            s_prefix = prefix;
            if (tile == ntiles - 1) ctr->n_next = prefix + agg;
        }
        __syncthreads();
        int run = s_prefix + excl;
        for (int q = 0; q < kScanItems; ++q) {
            int idx = base + q;
            if (idx < total) s.cscan[idx] = run;
            run += vals[q];
        }
    }
}

// ---------------------------------------------------------------------------
// k_scatter: survivors to their new slot; movers stage their sort keys
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_scatter(Veh in, Veh out, Scratch s, Counters* ctr) {
    const int N = ctr->n;
    const int M = ctr->nmove;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N + M; i += gridDim.x * kBlock) {
        if (i < N) {
            if (!s.stay[i]) continue;
            const int j = s.cscan[i] + s.mcnt[i];
            out.key[j] = in.key[i];
            out.x[j] = s.xs[i];
            out.v[j] = s.vs[i];
            out.edge[j] = in.edge[i];
            out.rcur[j] = in.rcur[i];
            out.next[j] = in.next[i];
            out.lc[j] = in.lc[i];
            out.kin[j] = in.kin[i];
            out.phin[j] = in.phin[i];
            out.vid[j] = in.vid[i];
        } else {
            const int m = i - N;
            const int p = s.mv_p[m];
            const int ci = s.mv_claim[m];
            const int b = s.cscan[p];
            s.mv_g[m] = s.mcnt[p];
            s.grp_key[b + s.mv_slot[m]] = s.cl_key[ci];
            s.grp_X[b + s.mv_slot[m]] = s.cl_X[ci];
        }
    }
}

// ---------------------------------------------------------------------------
// k_place: movers take their rank inside their gap; last block finalises
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_place(Trips tr, Veh in, Veh out, Scratch s, int lc_none,
                                                  Counters* ctr) {
    const int t = ctr->t;
    const int M = ctr->nmove;
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < M; m += gridDim.x * kBlock) {
        const int ci = s.mv_claim[m];
        const int p = s.mv_p[m];
        const int b = s.cscan[p];
        const int g = s.mv_g[m];
        const int key = s.cl_key[ci];
        const float X = s.cl_X[ci];
        int r = 0;
        if (g > 1) {
            for (int q = 0; q < g; ++q) {
                int kq = s.grp_key[b + q];
                if (kq < key || (kq == key && s.grp_X[b + q] < X)) ++r;
            }
        }
        const int j = b + r;
        const int kind = s.cl_kind[ci];
        const int src = s.cl_src[ci];
        const int vid = s.cl_vid[ci];
        out.key[j] = key;
        out.x[j] = X;
        out.v[j] = s.cl_v[ci];
        out.edge[j] = s.cl_tedge[ci];
        out.vid[j] = vid;
        if (kind == kCross) {
            const int rc = in.rcur[src] + 1;
            out.rcur[j] = rc;
            out.next[j] = (rc + 1 < tr.rend[vid]) ? tr.route_edges[rc + 1] : -1;
            out.lc[j] = in.lc[src];
            out.kin[j] = t + 1;
            out.phin[j] = s.cl_f[ci];
        } else if (kind == kChange) {
            out.rcur[j] = in.rcur[src];
            out.next[j] = in.next[src];
            out.lc[j] = t;
            out.kin[j] = in.kin[src];
            out.phin[j] = in.phin[src];
        } else {
            const int rc = tr.rbeg[vid];
            out.rcur[j] = rc;
            out.next[j] = (rc + 1 < tr.rend[vid]) ? tr.route_edges[rc + 1] : -1;
            out.lc[j] = lc_none;
            out.kin[j] = t + 1;
            out.phin[j] = 1.0f;
        }
        s.mcnt[p] = 0;
    }
    // last block to finish advances the step
    __syncthreads();
    __shared__ bool last;
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned prev = atomicAdd(&ctr->done_blocks, 1u);
        last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        ctr->updates += (unsigned long long)ctr->n;
        ctr->claims += (unsigned long long)ctr->nclaim;
        ctr->n = ctr->n_next;
        ctr->npend = ctr->npend_next;
        ctr->npend_next = 0;
        ctr->nclaim = 0;
        ctr->nmove = 0;
        ctr->done_blocks = 0;
        ctr->t = t + 1;
    }
}

__global__ void k_fill_u64(unsigned long long* p, long long n, unsigned long long v) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = v;
}

}  // namespace

// ===========================================================================
// host side
// ===========================================================================
struct sim_t {
    hipStream_t stream = nullptr;
    sim_alloc_fn alloc = nullptr;
    sim_free_fn free_fn = nullptr;
    void* ctx = nullptr;
    std::string err;
    std::vector<void*> allocs;

    int nn = 0, ne = 0, nlanes = 0, ncls = 0;
    std::vector<int> row_ptr, col_idx, lanes, cls, lane_base, ncell;
    std::vector<float> len, speed;
    long long ncells = 0;

    Params P{};
    Net net{};
    Trips tr{};
    Veh buf[2]{};
    Scratch s{};
    int* pend[2]{nullptr, nullptr};
    Counters* ctr = nullptr;
    float* d_inv_v0 = nullptr;
    float* d_cT = nullptr;
    float* d_cA = nullptr;
    float* d_cKab = nullptr;

    bool loaded = false;
    int cap = 0;
    int ntrips = 0;
    long long host_t = 0;  // steps enqueued so far (selects the buffer parity)
    int grid = 1;
    std::vector<int> h_rbeg;
    int timing_every = 0;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::vector<hipEvent_t>> ev_steps;  // SIM_NUM_KERNELS + 1 events per sampled step
};

namespace {

int fail(sim_t* S, int code, const std::string& msg) {
    if (S) S->err = msg;
    return code;
}

#define HIPCHECK(S, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((S), SIM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));        \
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

void release_all(sim_t* S) {
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    else (void)hipDeviceSynchronize();
    for (void* p : S->allocs) {
        if (S->free_fn) S->free_fn(S->ctx, p);
        else (void)hipFree(p);
    }
    S->allocs.clear();
}

int upload_idm(sim_t* S, const float* idm) {
    std::vector<float> T(S->ncls), A(S->ncls), K(S->ncls), inv(S->ne);
    for (int c = 0; c < S->ncls; ++c) {
        double s0 = idm[4 * c + 0], t = idm[4 * c + 1], a = idm[4 * c + 2], b = idm[4 * c + 3];
        if (!(s0 > 0) || !(t >= 0) || !(a > 0) || !(b > 0) || !std::isfinite(s0 * t * a * b))
            return fail(S, SIM_EINVAL, "idm parameters of class " + std::to_string(c) + " out of range");
        T[c] = (float)t;
        A[c] = (float)a;
        K[c] = (float)(1.0 / (2.0 * std::sqrt(a * b)));
    }
    for (int e = 0; e < S->ne; ++e)
        inv[e] = (float)(1.0 / ((double)idm[4 * S->cls[e] + 0] * (double)S->speed[e]));
    HIPCHECK(S, hipMemcpyAsync(S->d_cT, T.data(), sizeof(float) * S->ncls, hipMemcpyHostToDevice, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_cA, A.data(), sizeof(float) * S->ncls, hipMemcpyHostToDevice, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_cKab, K.data(), sizeof(float) * S->ncls, hipMemcpyHostToDevice, S->stream));
    HIPCHECK(S, hipMemcpyAsync(S->d_inv_v0, inv.data(), sizeof(float) * S->ne, hipMemcpyHostToDevice, S->stream));
    HIPCHECK(S, hipStreamSynchronize(S->stream));
    return SIM_OK;
}

template <class T>
int h2d(sim_t* S, T* dst, const T* src, size_t n) {
    if (n == 0) return SIM_OK;
    HIPCHECK(S, hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyHostToDevice, S->stream));
    return SIM_OK;
}

int32_t tail_node(const sim_t* S, int32_t e) {
    // largest u with row_ptr[u] <= e
    auto it = std::upper_bound(S->row_ptr.begin(), S->row_ptr.end(), e);
    return (int32_t)(it - S->row_ptr.begin()) - 1;
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
    if (nn <= 0 || ne <= 0 || ncls <= 0 || ncls > 4096) return SIM_EINVAL;
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

    float *d_len, *dummy;
    int *d_lane_base, *d_lanes, *d_cls, *d_head, *d_row_ptr, *d_ncell;
    long long* d_cbase;
    bool ok = dalloc(S, d_len, ne) && dalloc(S, S->d_inv_v0, ne) && dalloc(S, d_lane_base, ne + 1) &&
              dalloc(S, d_lanes, ne) && dalloc(S, d_cls, ne) && dalloc(S, d_head, ne) &&
              dalloc(S, d_row_ptr, nn + 1) && dalloc(S, d_cbase, ne) && dalloc(S, d_ncell, ne) &&
              dalloc(S, S->d_cT, ncls) && dalloc(S, S->d_cA, ncls) && dalloc(S, S->d_cKab, ncls) &&
              dalloc(S, S->s.cells, (size_t)cells) && dalloc(S, S->s.st_cnt, ne) &&
              dalloc(S, S->s.st_steps, ne) && dalloc(S, S->s.st_us, ne) && dalloc(S, S->ctr, 1) &&
              dalloc(S, dummy, 1);
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
    if ((rc = upload_idm(S, prm->idm)) != SIM_OK) {
        release_all(S);
        delete S;
        return rc;
    }
    hipError_t he = hipMemsetAsync(S->s.st_cnt, 0, sizeof(unsigned long long) * ne, S->stream);
    if (he == hipSuccess) he = hipMemsetAsync(S->s.st_steps, 0, sizeof(unsigned long long) * ne, S->stream);
    if (he == hipSuccess) he = hipMemsetAsync(S->s.st_us, 0, sizeof(unsigned long long) * ne, S->stream);
    if (he == hipSuccess) he = hipMemsetAsync(S->ctr, 0, sizeof(Counters), S->stream);
    if (he == hipSuccess) {
        int g = (int)std::min<long long>(kMaxGrid, std::max<long long>(1, (cells + kBlock - 1) / kBlock));
        hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(kBlock), 0, S->stream, S->s.cells, cells, ~0ull);
        he = hipGetLastError();
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
    std::vector<int> rbeg(ntrips), rend(ntrips), dep(ntrips);
    for (int v = 0; v < ntrips; ++v) {
        int i = ord[v];
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
    std::vector<unsigned char> placed(ntrips, init_x ? 1 : 0);
    // placed vehicles: validated, then sorted by (lane, position)
    std::vector<int> pkey, pedge, prcur, pnext, plc, pkin, pvid;
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
            if (key[a] == key[b] && ((init_x[ord[b]] - S->P.lveh) - init_x[ord[a]]) < 0.0f)
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
        }
    }

    const int cap = std::max(ntrips, 1);
    S->cap = cap;
    S->ntrips = ntrips;
    int* d_re;
    int *d_rbeg, *d_rend, *d_rel;
    unsigned char* d_placed;
    Scratch& s = S->s;
    bool ok = dalloc(S, d_re, (size_t)nre) && dalloc(S, d_rbeg, cap) && dalloc(S, d_rend, cap) &&
              dalloc(S, d_rel, rel_len + 1) && dalloc(S, d_placed, cap) &&
              dalloc(S, S->tr.depart_actual, cap) && dalloc(S, S->tr.arrive_step, cap) &&
              dalloc(S, S->pend[0], cap) && dalloc(S, S->pend[1], cap);
    for (int b = 0; b < 2 && ok; ++b) {
        Veh& V = S->buf[b];
        ok = dalloc(S, V.key, cap) && dalloc(S, V.x, cap) && dalloc(S, V.v, cap) && dalloc(S, V.edge, cap) &&
             dalloc(S, V.rcur, cap) && dalloc(S, V.next, cap) && dalloc(S, V.lc, cap) &&
             dalloc(S, V.kin, cap) && dalloc(S, V.phin, cap) && dalloc(S, V.vid, cap);
    }
    const size_t ntiles = (size_t)(cap + 1 + kScanTile - 1) / kScanTile + 1;
    ok = ok && dalloc(S, s.xs, cap) && dalloc(S, s.vs, cap) && dalloc(S, s.stay, cap + 1) &&
         dalloc(S, s.mcnt, cap + 1) && dalloc(S, s.cscan, cap + 1) && dalloc(S, s.cl_vid, cap) &&
         dalloc(S, s.cl_key, cap) && dalloc(S, s.cl_lo, cap) && dalloc(S, s.cl_hi, cap) &&
         dalloc(S, s.cl_src, cap) && dalloc(S, s.cl_kind, cap) && dalloc(S, s.cl_tedge, cap) &&
         dalloc(S, s.cl_X, cap) && dalloc(S, s.cl_v, cap) && dalloc(S, s.cl_f, cap) &&
         dalloc(S, s.mv_claim, cap) && dalloc(S, s.mv_p, cap) && dalloc(S, s.mv_slot, cap) &&
         dalloc(S, s.mv_g, cap) && dalloc(S, s.grp_key, cap) && dalloc(S, s.grp_X, cap) &&
         dalloc(S, s.tile_status, ntiles);
    if (!ok) return fail(S, SIM_ENOMEM, "device allocation failed in sim_load_demand");
    int rc;
    std::vector<int> minus1(cap, -1);
    if ((rc = h2d(S, d_re, route_edges, (size_t)nre)) || (rc = h2d(S, d_rbeg, rbeg.data(), ntrips)) ||
        (rc = h2d(S, d_rend, rend.data(), ntrips)) || (rc = h2d(S, d_rel, rel.data(), rel_len + 1)) ||
        (rc = h2d(S, d_placed, placed.data(), ntrips)) ||
        (rc = h2d(S, S->tr.arrive_step, minus1.data(), cap)))
        return rc;
    std::vector<int> da(cap, init_x ? t0 : -1);
    if ((rc = h2d(S, S->tr.depart_actual, da.data(), cap))) return rc;
    HIPCHECK(S, hipMemsetAsync(s.mcnt, 0, sizeof(int) * (cap + 1), S->stream));
    HIPCHECK(S, hipMemsetAsync(s.stay, 0, cap + 1, S->stream));
    HIPCHECK(S, hipMemsetAsync(s.tile_status, 0, sizeof(unsigned long long) * ntiles, S->stream));
    const int p = (int)(S->host_t & 1);
    const int np = (int)pkey.size();
    if (np) {
        Veh& V = S->buf[p];
        if ((rc = h2d(S, V.key, pkey.data(), np)) || (rc = h2d(S, V.x, px.data(), np)) ||
            (rc = h2d(S, V.v, pv.data(), np)) || (rc = h2d(S, V.edge, pedge.data(), np)) ||
            (rc = h2d(S, V.rcur, prcur.data(), np)) || (rc = h2d(S, V.next, pnext.data(), np)) ||
            (rc = h2d(S, V.lc, plc.data(), np)) || (rc = h2d(S, V.kin, pkin.data(), np)) ||
            (rc = h2d(S, V.phin, pphin.data(), np)) || (rc = h2d(S, V.vid, pvid.data(), np)))
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
    S->tr.placed = d_placed;
    S->h_rbeg = rbeg;
    S->grid = (int)std::min<long long>(kMaxGrid, std::max<long long>(1, ((long long)cap + kBlock - 1) / kBlock));
    S->loaded = true;
    return SIM_OK;
}

int sim_step(sim_t* S, int32_t num_steps) {
    if (!S) return SIM_EINVAL;
    if (!S->loaded) return fail(S, SIM_ESTATE, "no demand loaded");
    if (num_steps < 0) return fail(S, SIM_EINVAL, "negative step count");
    const dim3 g(S->grid), b(kBlock);
    for (int k = 0; k < num_steps; ++k) {
        const int p = (int)(S->host_t & 1);
        const Veh& in = S->buf[p];
        const Veh& out = S->buf[p ^ 1];
        int* pin = S->pend[p];
        int* pout = S->pend[p ^ 1];
        hipEvent_t ev[SIM_NUM_KERNELS + 1] = {};
        const bool timed = S->timing_every > 0 && (S->host_t % S->timing_every) == 0;
        if (timed) {
            for (int q = 0; q <= SIM_NUM_KERNELS; ++q) {
                if (S->ev_free.empty()) {
                    hipEvent_t e;
                    HIPCHECK(S, hipEventCreate(&e));
                    S->ev_free.push_back(e);
                }
                ev[q] = S->ev_free.back();
                S->ev_free.pop_back();
            }
            HIPCHECK(S, hipEventRecord(ev[0], S->stream));
        }
        hipLaunchKernelGGL(k_decide, g, b, 0, S->stream, S->P, S->net, S->tr, in, S->s, pin, pout, S->ctr);
        if (timed) HIPCHECK(S, hipEventRecord(ev[1], S->stream));
        hipLaunchKernelGGL(k_resolve, g, b, 0, S->stream, S->P, S->net, S->tr, in, S->s, pout, S->ctr);
        if (timed) HIPCHECK(S, hipEventRecord(ev[2], S->stream));
        hipLaunchKernelGGL(k_scan, g, b, 0, S->stream, S->s, S->ctr);
        if (timed) HIPCHECK(S, hipEventRecord(ev[3], S->stream));
        hipLaunchKernelGGL(k_scatter, g, b, 0, S->stream, in, out, S->s, S->ctr);
        if (timed) HIPCHECK(S, hipEventRecord(ev[4], S->stream));
        hipLaunchKernelGGL(k_place, g, b, 0, S->stream, S->tr, in, out, S->s, kLcNone, S->ctr);
        if (timed) {
            HIPCHECK(S, hipEventRecord(ev[5], S->stream));
            S->ev_steps.emplace_back(ev, ev + SIM_NUM_KERNELS + 1);
        }
        HIPCHECK(S, hipGetLastError());
        S->host_t += 1;
    }
    return SIM_OK;
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
    }
    return SIM_OK;
}

int sim_read_vehicles(sim_t* S, int32_t cap, int32_t* n_out, int32_t* vid, int32_t* edge, int32_t* lane,
                      int32_t* cursor, int32_t* lc, int32_t* kin, float* x, float* v, float* phin) {
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
    std::vector<int> hvid(n), hedge(n), hkey(n), hrcur(n);
    if (n) {
        HIPCHECK(S, hipMemcpyAsync(hvid.data(), V.vid, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipMemcpyAsync(hedge.data(), V.edge, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipMemcpyAsync(hkey.data(), V.key, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipMemcpyAsync(hrcur.data(), V.rcur, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        if (lc) HIPCHECK(S, hipMemcpyAsync(lc, V.lc, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        if (kin) HIPCHECK(S, hipMemcpyAsync(kin, V.kin, sizeof(int) * n, hipMemcpyDeviceToHost, S->stream));
        if (x) HIPCHECK(S, hipMemcpyAsync(x, V.x, sizeof(float) * n, hipMemcpyDeviceToHost, S->stream));
        if (v) HIPCHECK(S, hipMemcpyAsync(v, V.v, sizeof(float) * n, hipMemcpyDeviceToHost, S->stream));
        if (phin) HIPCHECK(S, hipMemcpyAsync(phin, V.phin, sizeof(float) * n, hipMemcpyDeviceToHost, S->stream));
        HIPCHECK(S, hipStreamSynchronize(S->stream));
    }
    for (int i = 0; i < n; ++i) {
        if (vid) vid[i] = hvid[i];
        if (edge) edge[i] = hedge[i];
        if (lane) lane[i] = hkey[i] - S->lane_base[hedge[i]];
        if (cursor) cursor[i] = hrcur[i] - S->h_rbeg[hvid[i]];
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

int sim_set_idm(sim_t* S, const float* idm) {
    if (!S || !idm) return SIM_EINVAL;
    return upload_idm(S, idm);
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
            HIPCHECK(S, hipEventElapsedTime(&ms, evs[q], evs[q + 1]));
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
    release_all(S);
    for (auto& evs : S->ev_steps)
        for (hipEvent_t e : evs) S->ev_free.push_back(e);
    for (hipEvent_t e : S->ev_free) (void)hipEventDestroy(e);
    delete S;
}

}  // extern "C"
