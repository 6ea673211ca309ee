// Validation of a simulation state against what the step kernels assume of
// it (included once, by trafficsim.hip).  The step indexes link, lane, route,
// trip and queue arrays with the values a state holds (lane keys, links,
// vehicle ids, types, route cursors, queue heads), and it takes the vehicles
// of a lane to be consecutive entries ordered by position; a state image
// handed in from outside is checked against all of that before any of it is
// copied in, and a running simulation can be checked at any step.  Each check
// tests its index before it uses it, so the pass itself stays in bounds on
// any input.
#pragma once

#include "common.h"

namespace tsim {

// classes of violations, in the order of the public sim_check_class enum
enum : int {
    kChkCount = 0,  // vehicle count outside [0, capacity] or a negative step
    kChkKey,        // lane key outside [0, lanes)
    kChkEdge,       // link outside [0, links) or the lane key not one of its lanes
    kChkOrder,      // entries not ordered by (lane key, position)
    kChkPos,        // position not finite or negative
    kChkSpeed,      // speed not finite or negative
    kChkVid,        // vehicle id outside [0, trips)
    kChkDup,        // a vehicle id on the road twice
    kChkType,       // vehicle type outside [0, types) or not the trip's type
    kChkRoute,      // route cursor outside the trip's route, or the route's link there not the vehicle's
    kChkNext,       // next link not the route's next one (-1 after the last)
    kChkValue,      // entry fraction outside [0, 1], fuel or CO not finite
    kChkArrived,    // a vehicle on the road whose trip has an arrival step
    kChkQueue,      // a departure queue's head after its tail, or its tail past its trips
    kChkHolder,     // a stop node's holder neither -1 nor a vehicle id
    kChkClasses
};

// the arrays of one state: the sorted vehicles (n entries), their trip state
// and arrival steps by vehicle id, the departure queues, the stop-node holders
struct CheckIn {
    const int* key;
    const float* x;
    const float* v;
    const int* edge;
    const int* next;
    const int* vid;
    const float* fuel;
    const float* co;
    const unsigned char* ty;
    const int* rcur;
    const float* phin;
    const int* arrive;
    const int* qstate;  // heads [0, nq), then tails [nq, 2 nq)
    const int* holder;
    int n;
};

__device__ __forceinline__ void check_fail(unsigned long long* fails, int* first, int cls, int at) {
    atomicAdd(fails + cls, 1ull);
    atomicMin(first + cls, at);
}

// One pass over the vehicles, the queues and the stop nodes.  seen holds a
// bit per vehicle id, zero on entry; fails and first (kChkClasses each) hold
// 0 and INT_MAX on entry and receive the count and the lowest offending entry
// (vehicle entry, queue or node) of every class.
__global__ void k_check_state(CheckIn c, Net net, Trips tr, int nlanes, int nt, int ntrips, int nn,
                              unsigned* seen, unsigned long long* fails, int* first) {
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < c.n; i += stride) {
        const int k = c.key[i], e = c.edge[i], nx = c.next[i], id = c.vid[i], ty = c.ty[i];
        const float x = c.x[i], v = c.v[i];
        if (k < 0 || k >= nlanes) check_fail(fails, first, kChkKey, i);
        const bool eok = 0 <= e && e < net.ne;
        bool kon = false;
        if (eok) {
            const int lb = net.lane_base[e];
            kon = lb <= k && k < lb + net.lanes[e];
        }
        if (!kon) check_fail(fails, first, kChkEdge, i);
        if (i + 1 < c.n) {
            const int k2 = c.key[i + 1];
            const float x2 = c.x[i + 1];
            if (!(k < k2 || (k == k2 && x <= x2))) check_fail(fails, first, kChkOrder, i);
        }
        if (!__builtin_isfinite(x) || x < 0.0f) check_fail(fails, first, kChkPos, i);
        if (!__builtin_isfinite(v) || v < 0.0f) check_fail(fails, first, kChkSpeed, i);
        const bool vok = 0 <= id && id < ntrips;
        if (!vok) {
            check_fail(fails, first, kChkVid, i);
        } else {
            const unsigned bit = 1u << (id & 31);
            if (atomicOr(seen + (id >> 5), bit) & bit) check_fail(fails, first, kChkDup, i);
        }
        if (ty >= nt || (vok && ty != (int)tr.vtype[id])) check_fail(fails, first, kChkType, i);
        bool vals = __builtin_isfinite(c.fuel[i]) && __builtin_isfinite(c.co[i]);
        if (vok) {
            const int rc = c.rcur[id], rb = tr.rbeg[id], re = tr.rend[id];
            if (rc < rb || rc >= re || !eok || tr.route_edges[rc] != e) {
                check_fail(fails, first, kChkRoute, i);
            } else {
                const int want = rc + 1 < re ? tr.route_edges[rc + 1] : -1;
                if (nx != want) check_fail(fails, first, kChkNext, i);
            }
            const float ph = c.phin[id];
            vals = vals && ph >= 0.0f && ph <= 1.0f;
            if (c.arrive[id] >= 0) check_fail(fails, first, kChkArrived, i);
        }
        if (!vals) check_fail(fails, first, kChkValue, i);
    }
    for (int q = blockIdx.x * kBlock + threadIdx.x; q < tr.nq; q += stride) {
        const int h = c.qstate[q], tl = c.qstate[tr.nq + q];
        if (h < 0 || h > tl || tl > tr.qoff[q + 1] - tr.qoff[q]) check_fail(fails, first, kChkQueue, q);
    }
    for (int h = blockIdx.x * kBlock + threadIdx.x; h < nn; h += stride) {
        const int hd = c.holder[h];
        if (hd != -1 && (hd < 0 || hd >= ntrips)) check_fail(fails, first, kChkHolder, h);
    }
}

}  // namespace tsim
