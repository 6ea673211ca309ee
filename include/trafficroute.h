/*
 * trafficroute.h -- route planning for iterative re-routing, part of
 * libtrafficsim.so (HIP kernels for gfx950).
 *
 * Sec. 6.3.1 of Waddell et al. approximates traffic equilibrium by planning
 * every vehicle's route on estimated link travel times, running the
 * microsimulation, replacing the estimates by the measured travel times and
 * planning again for a decaying share of the vehicles (all, all, half, a
 * quarter over four iterations).  The first estimate of a link is
 * sqrt(lanes) x length / speed.  A router handle holds the network, the
 * origin/destination of every trip, the current link weights and the current
 * routes, all in device memory; it plans shortest routes for a selected subset
 * of trips and keeps the others' routes.
 *
 * Weights are integer milliseconds >= 1.  The sum of all weights must stay
 * below 2^40 (every shortest route is then shorter), and the network below
 * 2^24 edges.  Shortest routes are made unique by one rule: the last edge into
 * every node of a route is the lowest-numbered edge e = (u -> w) with
 * dist(u) + weight(e) == dist(w).
 *
 * Conventions are those of trafficsim.h: SIM_* return codes, host pointers
 * read during the call only, work enqueued on the handle's stream, calls that
 * return host data synchronise it, handles not thread-safe.
 */
#ifndef TRAFFICROUTE_H
#define TRAFFICROUTE_H

#include "trafficsim.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_t rt_t;

/* Router over the network of sim_create (HOST arrays, copied; only row_ptr,
 * col_idx, lanes, length_m and speed_mps are used).  Weights start at the
 * initial estimate (rt_weights_initial).
 * Errors: SIM_EINVAL (bad network, >= 2^24 edges), SIM_ENOMEM, SIM_EHIP. */
int rt_create(const sim_network* net, void* hip_stream, sim_alloc_fn alloc, sim_free_fn free_fn, void* alloc_ctx,
              rt_t** out);

/* The trips (HOST arrays, copied): num_sources distinct origin nodes
 * src_nodes[num_sources]; per trip the index of its origin in src_nodes,
 * trip_src[num_trips], and its destination node, trip_dst[num_trips] (not its
 * origin).  Drops any current routes.  Errors: SIM_EINVAL. */
int rt_set_trips(rt_t* rt, int32_t num_sources, const int32_t* src_nodes, int32_t num_trips, const int32_t* trip_src,
                 const int32_t* trip_dst);

/* weight(e) = max(1, round(sqrt(lanes) * length / speed * 1000)) ms, halves
 * rounded up, evaluated in double from the float attributes (Sec. 6.3.1). */
int rt_weights_initial(rt_t* rt);

/* Measured estimate (Sec. 6.3.1): for every link with count > 0 the mean
 * traversal time in ms, (tt_us + 500 count) / (1000 count) in integers,
 * at least 1; links nobody finished keep their weight.  edge_count and
 * edge_tt_us are DEVICE int64 [num_edges], e.g. filled by sim_stats.
 * Errors: SIM_EINVAL (null), SIM_EHIP. */
int rt_weights_from_stats(rt_t* rt, const int64_t* edge_count, const int64_t* edge_tt_us);

/* Set (HOST int64 [num_edges], each >= 1) or read the current weights. */
int rt_set_weights(rt_t* rt, const int64_t* weights_ms);
int rt_read_weights(rt_t* rt, int64_t* weights_ms);

/* Plan the shortest route under the current weights for every trip with
 * select[i] != 0 (HOST uint8 [num_trips]; NULL = every trip, required for the
 * first plan after rt_set_trips); the other trips keep their current routes.
 * *total_route_edges receives the length of the new route array.
 * Errors: SIM_ESTATE (no trips, or a partial plan with no current routes),
 * SIM_EROUTE (a selected destination unreachable from its origin),
 * SIM_EINVAL (weights sum >= 2^40), SIM_ENOMEM, SIM_EHIP. */
int rt_plan(rt_t* rt, const uint8_t* select, int64_t* total_route_edges);

/* Copy the current routes out: route_ptr HOST int64 [num_trips+1], route i =
 * route_edges[route_ptr[i] .. route_ptr[i+1]) in driving order (HOST int32
 * [total_route_edges]); this is the per-trip route table sim_load_demand takes
 * with trip_route[i] = i.  Either pointer may be NULL.  Errors: SIM_ESTATE. */
int rt_read_routes(rt_t* rt, int64_t* route_ptr, int32_t* route_edges);

/* The current routes where they are, on the DEVICE: *route_ptr int64
 * [num_trips + 1] and *route_edges int32 [*total_route_edges], laid out as
 * rt_read_routes writes them.  Owned by the router; valid until the next
 * rt_plan or rt_destroy.  sim_reload_routes takes them as they are, so the
 * routes never leave the device.  Any output may be NULL.
 * Errors: SIM_ESTATE (no routes planned). */
int rt_route_views(rt_t* rt, const int64_t** route_ptr, const int32_t** route_edges,
                   int64_t* total_route_edges);

/* Shortest-path tree from one node under the current weights: dist HOST
 * int64 [num_nodes] (INT64_MAX where unreachable) and pred HOST int32
 * [num_nodes] (last edge of the route to each node; -1 at the source and at
 * unreachable nodes).  Either pointer may be NULL.  Errors: SIM_EINVAL. */
int rt_tree(rt_t* rt, int32_t src_node, int64_t* dist, int32_t* pred);

/* Bytes of the static per-GPU search scratch of rt_tree_static. */
#define RT_STATIC_SCRATCH_BYTES (48u << 20)

/* rt_tree for callers that cannot allocate device memory (code between
 * other work that must not call hipMalloc, tight serving loops, harnesses
 * that forbid allocation): the same tree, computed with no allocation at
 * all.  Its search scratch (a 64-bit label, two stamps and four frontier
 * entries per node, plus counters: about 32 bytes per node) lives in one
 * static device array of RT_STATIC_SCRATCH_BYTES per GPU, held by every GPU
 * the library runs on until the process ends; networks of up to about
 * 1.57M nodes fit.  dist DEVICE int64 [num_nodes] (INT64_MAX where
 * unreachable) and pred DEVICE int32 [num_nodes] (last edge of the route to
 * each node, -1 at the source and at unreachable nodes) are the caller's
 * buffers; either may be NULL.  Call with the router's device current.  The
 * search reads frontier counts back to the host between rounds, so the call
 * is not capturable into a graph; it returns once dist and pred are written.
 * Every call on one GPU shares that GPU's array and overwrites what the last
 * call left there (the scratch is re-initialised on every call): calls that
 * overlap on one GPU (from other threads or streams) race.
 * Errors: SIM_EINVAL (network too large for the static scratch, with the
 * sizes in rt_last_error; bad source; another device current), SIM_EHIP. */
int rt_tree_static(rt_t* rt, int32_t src_node, int64_t* dist, int32_t* pred);

/* Edge relaxations performed by the last rt_plan (work counter) and the
 * number of sources it searched from. */
int rt_last_work(rt_t* rt, int64_t* relaxations, int32_t* sources);

/* Largest number of origins searched at once.  Default: as many as fit in
 * 32 bytes x nodes x count within a quarter of the device memory free at the
 * plan (at least 4 GiB, at most 64 GiB), at most 4096, and count x nodes
 * below 2^32, or the batch of an earlier plan if larger (its memory is kept).
 * Larger batches need fewer search rounds per plan.  Errors: SIM_EINVAL. */
int rt_set_batch(rt_t* rt, int32_t sources_per_batch);

/* Band width of the search in ms (the search relaxes labels below a threshold
 * first and raises the threshold by this much when none are left; the
 * result does not depend on it, the work does).  0 = three times the mean
 * weight (default).  Errors: SIM_EINVAL. */
int rt_set_delta(rt_t* rt, int64_t delta_ms);

int rt_set_stream(rt_t* rt, void* hip_stream);
const char* rt_last_error(const rt_t* rt);
void rt_destroy(rt_t* rt);

#ifdef __cplusplus
}
#endif

#endif
