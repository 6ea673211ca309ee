// Device-side data structures and helpers shared by the step kernels and the
// adjoint kernels of libtrafficsim (included once, by trafficsim.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tsim {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kScanItems = 32;
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kLcNone = -(1 << 30);
constexpr int kMaxGrid = 2048;
// k_decide's largest tile of sorted entries (block size x entries per thread);
// a claim segment holds one eighth of the tiles of this size
constexpr int kMaxTile = 1024;
// A list that every wave of a step may append to (lane-change candidates,
// claims) is split into kSeg segments with one counter each, in lines of their
// own.  Blocks are dispatched to the XCDs in turn, so block b runs on XCD
// b % kSeg: the vehicle blocks of XCD q take the q-th eighth of the sorted
// entries (in 256-entry chunks) and append to segment q, and departure queue
// chunk c (256 queues) appends to segment c % kSeg.  The appends of one XCD
// meet one counter and stay in its L2; one counter for the whole chip would
// serialise every wave's append.
constexpr int kSeg = 8;
constexpr int kSegStride = 32;  // ints from one segment counter to the next
// The step's statistics are summed the same way: one line of kStatStride
// counters per XCD (block b adds to line b % kSeg), folded into the Counters
// when the step ends.
enum : int { kStClamps = 0, kStArrived, kStGhost, kStLost, kStDepClaims, kStLcEval, kStLcClaims, kStDeparted };
constexpr int kStatStride = 16;
// Coarse index of the sorted keys: lanes are grouped in blocks of
// 2^kLaneBlkLog; lblk[b] is the first entry whose lane is in block b or later.
constexpr int kLaneBlkLog = 6;

enum : int { kCross = 1, kChange = 2, kInsert = 3 };

// ---------------------------------------------------------------------------
// device-side data
// ---------------------------------------------------------------------------
struct Counters {
    int t;           // current step
    int n;           // vehicles on the road (entries of the current buffer)
    int n_next;      // entries of the next buffer
    unsigned scan_tile;
    unsigned epoch_next;  // epoch of the next step (set during the step, committed at its end)
    unsigned long long arrived, departed, updates, claims_lost, clamps, claims;
    unsigned long long claims_dep;  // of which departures (those counted without an entry included)
    unsigned long long lc_eval;     // vehicles evaluated for a lane change
    unsigned long long claims_lc;   // lane-change claims
};

struct Params {
    float dt, h, lveh, s0, claim_len, s_eps, b_max, pol, athr, bsafe, dmand, dt_us_f;
    float mph;  // miles per hour per m/s
    int green;  // steps of green per signal movement
    float stop_dist, stop_speed;  // a vehicle within stop_dist of a stop line at <= stop_speed is waiting
    long long dt_us;
    int lc_cool;
    // vehicle types (Sec. 6.3.5): length and claim length (length + s0)
    int nt;
    float tlen[4], tclaim[4];
};

// Packed per-link records for the step's hot path (one 16-byte load each
// instead of a chain of dependent gathers); the plain arrays below hold the
// same values for the other kernels.
struct __align__(16) EdgeRec {
    float len;
    int lane_base;
    int lanes;
    int r0;  // first out-link of the head node
};
// Per (link, vehicle type): what a vehicle needs of its own link, in one
// 32-byte record (one cache line): the driver constants and the link fields.
struct __align__(32) DrvRec {
    float iv, A, T, kab;  // 1/v0, acceleration, time gap, 1/(2 sqrt(ab))
    float len;
    int lane_base;
    int lanes_m;          // lanes | (out-degree of the head node) << 16
    int r0;               // first out-link of the head node
};
struct __align__(16) ClaimRec {
    long long cbase;  // first claim cell of lane 0
    int ncell;        // cells per lane
    int m;            // out-degree of the head node
};

struct Net {
    const EdgeRec* er;
    const DrvRec* drv;
    const ClaimRec* cr;
    const float* len;
    const float* inv_v0;
    const int* lane_base;
    const int* lanes;
    const int* cls;
    const int* head;
    const int* row_ptr;
    const long long* cbase;  // first claim cell of lane 0 of the edge
    const int* ncell;        // cells per lane = floor(len) + 1
    int ne;                  // number of edges
    const int* ctrl;         // per node: 0 none, 1 stop, 2 signal; NULL = no control anywhere
    const int* in_rank;      // per edge: rank among the inbound links of its head node
    const int* in_deg;       // per node: number of inbound links
    const float* cT;
    const float* cA;
    const float* cKab;
    const float* cVs;  // v0 scale per class (adjoint chain rule)
    const float* cB;   // comfortable deceleration per class (adjoint chain rule)
    // cA, cKab are [class * nt + type], inv_v0 [edge * nt + type]; a type's
    // acceleration cap (capA) or speed cap (capV) cuts the dependence on the
    // class parameter it replaces
    const unsigned char* capA;
    const unsigned char* capV;
};

struct Trips {
    const int* route_edges;
    const int* rbeg;
    const int* rend;
    const int* rel_off;  // rel_off[t] = first vehicle id due at step >= t
    int rel_len;         // rel_off has rel_len + 1 entries
    const unsigned char* vtype;  // per vehicle id
    // Departure queues: the trips of one (first link, type), by vehicle id,
    // which is also their order of departure steps.  Queue q holds entries
    // [qoff[q], qoff[q+1]) of qvid / qdep; qtail[q] of them are due so far and
    // the first qhead[q] have entered the road.
    int nq;
    const int* qoff;
    const int* qvid;
    const int* qdep;
    const int* qedge;
    const unsigned char* qtype;
    int* qhead;
    int* qtail;
    int* depart_actual;
    int* arrive_step;
    float* fuel_total;  // per vehicle id, at arrival
    float* co_total;
    // The state of a vehicle on the road that changes only when it enters a
    // link, by vehicle id (the sorted arrays do not carry it, so the
    // per-step re-sort does not move it): its current link's index in the
    // route, the step it entered that link and the fraction of the step at
    // which it did.
    int* rcur;
    int* kin;
    float* phin;
};

// The vehicles on the road, sorted by (lane key, position): what the step
// reads or changes every step.
struct Veh {
    int* key;
    float* x;
    float* v;
    int* edge;
    int* next;
    int* lc;
    int* vid;
    float* fuel;  // accumulated fuel (mL)
    float* co;    // accumulated CO (g)
    unsigned char* ty;  // vehicle type
};

// Entries [lo, hi] of the sorted arrays are the vehicles of one lane, valid
// when ep equals the current step's epoch (so the table is never cleared).
// The rearmost vehicle's type, position and speed ride along, so a vehicle
// that looks ahead into the next link reads one record instead of four.
struct __align__(32) LaneIx {
    unsigned ep;
    int lo;
    int hi;
    int ty;   // rearmost vehicle (entry lo): type,
    float x;  // position
    float v;  // and speed
    int pad0, pad1;
};

__device__ __forceinline__ bool lane_range(const LaneIx* __restrict__ lanes, int key, unsigned ep, int& lo, int& hi) {
    const int4 w = *reinterpret_cast<const int4*>(lanes + key);
    lo = w.y;
    hi = w.z;
    return (unsigned)w.x == ep;
}

__device__ __forceinline__ bool lane_rear(const LaneIx* __restrict__ lanes, int key, unsigned ep, int& lo,
                                          float& x, float& v, int& ty) {
    const int4 w = *reinterpret_cast<const int4*>(lanes + key);
    const float4 r = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(lanes + key) + 16);
    lo = w.y;
    ty = w.w;
    x = r.x;
    v = r.y;
    return (unsigned)w.x == ep;
}

struct Scratch {
    int* ccnt;    // counters of the kSeg segments of the claim list (cl_*), kSegStride ints apart
    int cl_seg;   // entries per claim segment
    unsigned long long* sstat;  // kSeg lines of per-XCD statistics
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
    long long* cl_cell;  // first claim cell of the claim's target lane
    float* cl_X;
    float* cl_v;
    float* cl_f;
    // movers (winning claims), in kSeg segments of cl_seg entries: the winners
    // of claim segment q go to mover segment q
    int* mvcnt;  // segment counters, kSegStride ints apart
    int* tcnt;   // per segment, k_decide's next tile (kSegStride ints apart; cleared by k_resolve)
    int* mv_claim;
    int* mv_src;  // the claim's source entry (departures: -2 - queue) and vehicle id
    int* mv_vid;
    int* mv_rc;   // crossings and departures: the route cursor and next link after the move
    int* mv_nx;
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
    // sampler: every samp_every steps, per link vehicle count and speed sum
    // (micrometres per second), accumulated in groups of samp_group samples
    int samp_every, samp_group, samp_max;
    unsigned long long* samp_cnt;
    unsigned long long* samp_spd;
    int* holder;                    // per stop node: vehicle admitted into the intersection, or -1
    unsigned long long* stop_req;   // per stop node: lowest (epoch, id) waiting at the line
    unsigned* epoch;  // executed-step counter (claims, scan statuses, lane index are tagged with it)
    LaneIx* lanes;  // per global lane: first and last entry in the sorted arrays
    int* lblk;      // [nlblk + 1]: first entry of lane block b (lblk[nlblk] = entries)
    int nlblk;      // lane blocks
};

// Event tape of one step (recorded during the adjoint's recompute pass): the
// state and the discrete outcome of every entry of the sorted vehicle arrays.
enum : int { kModeStay = 0, kModeChange = 1, kModeYield = 2, kModeArrive = 3, kModeCross = 4 };
enum : int {
    kFHasLead = 1, kFLeadCross = 2, kFDynFloor = 4, kFSFloor = 8, kFAccFloor = 16, kFStop = 32,
    kFDxFloor = 64, kFClamp = 128, kFClampZero = 256, kFClampV = 512, kFFOne = 1024,
    kFVirtual = 2048  // the vehicle ahead is the stop line of a held movement
};

struct Tape {
    int on;
    float* x;               // position and speed at the step
    float* v;
    int* vid;
    int* edge;
    int* lead;              // entry index of the vehicle ahead for the own-lane motion, or -1
    int* clead;             // ... for the lane-change motion
    int* next;              // entry index at the next step, -1 if the vehicle left
    unsigned char* mode;
    unsigned short* flags;  // branch flags of the own-lane motion
    unsigned short* cflags; // ... of the lane-change motion
    int* n;                 // number of entries
};

struct Lead {
    int kind;  // 0 free road, 1 same link, 2 rearmost vehicle of the next link, 3 stop line
    float s;   // bumper-to-bumper gap
    float vl;  // speed of the vehicle ahead
    float xl;  // its position on its own link
    int idx;   // its entry index in the sorted arrays
    float ll;  // its length
};

__device__ __forceinline__ int lead_flags(const Lead& L) {
    if (L.kind == 0) return 0;
    return kFHasLead | (L.kind == 2 ? kFLeadCross : 0) | (L.kind == 3 ? kFVirtual : 0);
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fmx(float a, float b) { return a > b ? a : b; }
__device__ __forceinline__ float fmn(float a, float b) { return a < b ? a : b; }

// IDM (Sec. 6.3.2, car-following equation, exponent 4): dynamic part of the
// desired gap floored at 0, gap floored at s_eps, result floored at -b_max.
__device__ __forceinline__ float idm_acc_fl(const Params& P, float A, float T, float kab, float iv,
                                            float v, const Lead& L, int& fl) {
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
        if (0.0f > dyn) fl |= kFDynFloor;
        float ss = P.s0 + fmx(0.0f, dyn);
        if (!(L.s > P.s_eps)) fl |= kFSFloor;
        float q = ss / fmx(L.s, P.s_eps);
        acc = A * (fr - q * q);
    }
    if (!(acc > -P.b_max)) fl |= kFAccFloor;
    return fmx(acc, -P.b_max);
}

__device__ __forceinline__ float idm_acc(const Params& P, float A, float T, float kab, float iv,
                                         float v, const Lead& L) {
    int fl = 0;
    return idm_acc_fl(P, A, T, kab, iv, v, L, fl);
}

// ballistic update; stop inside the step when the speed would turn negative
__device__ __forceinline__ void kin_move_fl(const Params& P, float v, float acc, float& dx, float& vn,
                                            int& fl) {
    float vv = v + acc * P.dt;
    if (vv < 0.0f) {
        dx = (v * v) / (-2.0f * acc);
        vn = 0.0f;
        fl |= kFStop;
    } else {
        dx = v * P.dt + acc * P.h;
        vn = vv;
    }
    if (!(dx > 0.0f)) fl |= kFDxFloor;
    dx = fmx(dx, 0.0f);
}

__device__ __forceinline__ void kin_move(const Params& P, float v, float acc, float& dx, float& vn) {
    int fl = 0;
    kin_move_fl(P, v, acc, dx, vn, fl);
}

__device__ __forceinline__ int clamp_to_leader_fl(const Lead& L, float& dx, float& vn, int& fl) {
    if (L.kind != 0 && dx > L.s) {
        fl |= kFClamp;
        if (!(L.s > 0.0f)) fl |= kFClampZero;
        if (!(vn < L.vl)) fl |= kFClampV;
        dx = fmx(L.s, 0.0f);
        vn = fmn(vn, L.vl);
        return 1;
    }
    return 0;
}

__device__ __forceinline__ int clamp_to_leader(const Lead& L, float& dx, float& vn) {
    int fl = 0;
    return clamp_to_leader_fl(L, dx, vn, fl);
}

__device__ __forceinline__ Lead relead(float len, const Lead& L, float xf) {
    Lead R = L;
    if (L.kind == 1) R.s = (L.xl - L.ll) - xf;
    else if (L.kind == 2) R.s = (len - xf) + (L.xl - L.ll);
    else if (L.kind == 3) R.s = len - xf;
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

// Fuel and CO over one step (Sec. 6.3.4): fuel-consumption equation with v in
// m/s and the realized acceleration a = (v1 - v)/dt, bracket floored at 0,
// P_ea only while accelerating; CO equation with v in miles per hour.
__device__ __forceinline__ void emissions(const Params& P, float v, float v1, float& fuel, float& co) {
    const float a = (v1 - v) / P.dt;
    const float vm = v * P.mph;
    const float d = vm - 50.0f;
    const float c = -0.064f + 0.0056f * vm + 0.00026f * (d * d);
    const float pea = a > 0.0f ? (0.79296f * (a * a)) * v : 0.0f;
    float br = 0.269f * v + 0.0171f * (v * v) + 0.000672f * ((v * v) * v) + 1.680f * (a * v) + pea;
    br = fmx(br, 0.0f);
    const float f = 0.666f + 0.072f * br;
    fuel = fuel + f * P.dt;
    co = co + c * P.dt;
}

// Intersection control (Sec. 6.3.2): is the movement e -> nx held at the end of
// e this step?  A stop node holds everyone but the vehicle it admitted (the
// lowest id waiting at its line when it was free, requested at the end of the
// previous step); a signal gives movement (inbound rank i, outbound rank j) the
// green in phase i*m + j of its n*m phases, `green` steps each.
__device__ __forceinline__ bool movement_held(const Params& P, const Net& net, const Scratch& s, int e, int nx,
                                             int vid, int t, unsigned long long tag) {
    if (!net.ctrl || nx < 0) return false;
    const int h = net.head[e];
    const int c = net.ctrl[h];
    if (c == 1) {
        const int hd = s.holder[h];
        if (hd == vid) return false;
        if (hd == -1 && s.stop_req[h] == (tag | (unsigned)vid)) {
            s.holder[h] = vid;  // admitted now
            return false;
        }
        return true;
    }
    if (c == 2) {
        const int r0 = net.row_ptr[h];
        const int m = net.row_ptr[h + 1] - r0;
        const int phase = (t / P.green) % (net.in_deg[h] * m);
        return phase != net.in_rank[e] * m + (nx - r0);
    }
    return false;
}

__device__ __forceinline__ Lead stop_line_lead(float len, float x) {
    Lead L = {3, len - x, 0.0f, len, -1, 0.0f};
    return L;
}

// claims of a later executed step always beat those of an earlier one
__device__ __forceinline__ unsigned long long epoch_tag(unsigned epoch) {
    return (unsigned long long)(0xFFFFFFFFu - epoch) << 32;
}

// a per-type constant, picked from registers (the table lives in the kernel
// arguments; indexing it with a per-lane type would be a memory read)
// A per-type constant of the parameters (uniform over the launch), chosen by
// selects between the four values held in scalar registers.  The empty asm
// hides that the values are the array's elements: otherwise the compiler
// folds the selects into one vector load at a type-dependent address in the
// kernel arguments, a memory round trip after the type is known.
__device__ __forceinline__ float by_type(const float (&a)[4], int ty) {
    float a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
    asm("" : "+s"(a0), "+s"(a1), "+s"(a2), "+s"(a3));
    float r = a0;
    r = ty == 1 ? a1 : r;
    r = ty == 2 ? a2 : r;
    r = ty == 3 ? a3 : r;
    return r;
}

// cells [lo, hi] of a lane of nc cells that a front at X claims for type ty
__device__ __forceinline__ void claim_cells(const Params& P, int nc, int ty, float X, int& lo, int& hi) {
    int a = (int)floorf(X - by_type(P.tclaim, ty));
    int b = (int)floorf(X);
    lo = a < 0 ? 0 : a;
    hi = b > nc - 1 ? nc - 1 : b;
}

// A slot in a list filled through one shared counter: the lanes of a wave
// that reach this point together take consecutive slots with a single atomic
// (the order of the slots carries no meaning anywhere in the step).
__device__ __forceinline__ int wave_slot(int* counter) {
    const unsigned long long mask = __ballot(1);
    const int lane = (int)__lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader, kWave);
    return base + rank;
}

// adds v to statistic `what` of the calling block's line
__device__ __forceinline__ void seg_stat(const Scratch& s, int what, unsigned long long v) {
    if (v) atomicAdd(s.sstat + (blockIdx.x & (kSeg - 1)) * kStatStride + what, v);
}

// A claim on lane tlane of link tedge (claim record C, first global lane
// lane_base) takes its cells, then a slot in segment seg (the same for the
// whole wave) of the claim list.
__device__ __forceinline__ void push_claim(const Scratch& s, const ClaimRec& C, int lane_base, int seg,
                                           unsigned long long tag, int vid, int kind, int src, int tedge, int tlane,
                                           float X, float vc, float f, int lo, int hi) {
    const long long cb = C.cbase + (long long)tlane * C.ncell;
    unsigned long long* cell = s.cells + cb;
    const unsigned long long mine = tag | (unsigned)vid;
    for (int c = lo; c <= hi; ++c) atomicMin(cell + c, mine);
    const int ci = seg * s.cl_seg + wave_slot(s.ccnt + seg * kSegStride);
    s.cl_vid[ci] = vid;
    s.cl_key[ci] = lane_base + tlane;
    s.cl_lo[ci] = lo;
    s.cl_hi[ci] = hi;
    s.cl_src[ci] = src;
    s.cl_kind[ci] = kind;
    s.cl_tedge[ci] = tedge;
    s.cl_cell[ci] = cb;
    s.cl_X[ci] = X;
    s.cl_v[ci] = vc;
    s.cl_f[ci] = f;
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

}  // namespace tsim
