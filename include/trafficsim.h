/*
 * trafficsim.h -- C ABI of the MI355X traffic microsimulation library
 * (libtrafficsim.so, HIP kernels for gfx950).
 *
 * The library advances a population of vehicles over a lane-level road network
 * in synchronous time steps, as the GPU traffic microsimulator of Waddell et
 * al., "Architecture for Modular Microsimulation of Real Estate Markets and
 * Transportation", Sec. 6: every vehicle follows a precomputed route
 * (Sec. 6.3.1) and is updated each step by lane changing and car following
 * (Sec. 6.3.2, car-following equation = Intelligent Driver Model), with
 * departures from per-trip departure times (Sec. 6.2.2) and per-link travel
 * time statistics (Sec. 6.4).
 *
 * Conventions for every entry point:
 *   - Return value: SIM_OK (0) or a negative SIM_E* code.  The library never
 *     aborts; sim_last_error() names the offending item of the last failure.
 *   - Host pointers are read during the call only (the caller may free them on
 *     return).  Pointers documented as "device" must be device memory that is
 *     valid on the handle's stream.
 *   - All GPU work is enqueued on the handle's HIP stream.  Entry points that
 *     return host data synchronise that stream first.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef TRAFFICSIM_H
#define TRAFFICSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SIM_OK = 0,
    SIM_EINVAL = -1, /* null pointer, size or value out of range, overlapping placement */
    SIM_EROUTE = -2, /* empty route, edge id out of range, or consecutive edges not joined */
    SIM_ENOMEM = -3, /* device allocation failed */
    SIM_EHIP = -4,   /* a HIP runtime call failed; sim_last_error has hipGetErrorString */
    SIM_ESTATE = -5  /* call not valid now (e.g. demand loaded twice, departure in the past) */
};

typedef struct sim_t sim_t;

/* Device allocator hooks.  alloc returns device memory of `bytes` bytes (or
 * NULL); free releases it.  Both NULL: the library uses hipMalloc/hipFree. */
typedef void* (*sim_alloc_fn)(void* ctx, size_t bytes);
typedef void (*sim_free_fn)(void* ctx, void* ptr);

/* Road network (Sec. 6.2.1): directed multigraph in CSR form by tail node.
 * Edge id == CSR position.  All arrays are HOST memory.
 *   row_ptr   [num_nodes+1]  row_ptr[0] = 0, row_ptr[num_nodes] = num_edges,
 *                            non-decreasing, at most 32767 out-links per node
 *   col_idx   [num_edges]    head node of each edge (self-loops allowed)
 *   lanes     [num_edges]    1..8
 *   length_m  [num_edges]    >= veh_length + s0
 *   speed_mps [num_edges]    speed limit > 0; desired speed v0 = v0_scale[class]*speed
 *   link_class[num_edges]    0..num_classes-1, or NULL (all class 0)            */
typedef struct {
    int32_t num_nodes, num_edges;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* lanes;
    const float* length_m;
    const float* speed_mps;
    const int32_t* link_class;
} sim_network;

/* Model parameters.  dt: time step (s; Sec. 6.3.2 uses 0.5).  veh_length and
 * s0 (minimum gap) in m.  idm: HOST [num_classes][4] = {v0_scale, T, a, b} of
 * the car-following equation (Sec. 6.3.2), exponent fixed at 4.  s_eps floors
 * the gap in the IDM interaction term; b_max floors the acceleration.  MOBIL
 * politeness, threshold and safe braking for discretionary lane changes;
 * mand_dist: distance to the link end below which a vehicle outside the lanes
 * of its next turn changes lanes mandatorily (Sec. 6.3.2, lane changing);
 * lc_cooldown_steps: minimum steps between two changes of one vehicle.      */
typedef struct {
    float dt, veh_length, s0, s_eps, b_max;
    int32_t num_classes;
    const float* idm;
    float mobil_p, mobil_athr, mobil_bsafe, mand_dist;
    int32_t lc_cooldown_steps;
} sim_params;

/* Counters (Sec. 6.4 outputs).  vehicle_updates = sum over completed steps of
 * the vehicles on the road at the start of the step. */
typedef struct {
    int64_t step, loaded, waiting, en_route, arrived, departed;
    int64_t vehicle_updates, claims_lost, clamps;
    int64_t claims; /* claims issued (crossings, lane changes, departures) */
    int64_t claims_departure; /* of which departures: of several trips waiting to
                               * enter one link by the same lane, only the one with
                               * the lowest id can win; the others are counted
                               * (here and in claims_lost) without a claim record */
    int64_t lc_evaluated;       /* vehicles that passed the lane-change eligibility
                                 * test (multi-lane link, cool-down over, fully on
                                 * the link, not leaving it) and were evaluated */
    int64_t claims_lane_change; /* of the claims, lane changes */
} sim_stats_t;

/* Create a simulation of `net` with `params` on `hip_stream` (a hipStream_t,
 * NULL = default stream).  Validates and copies the network; derived
 * constants (1/v0 per edge, 1/(2 sqrt(ab)) per class, dt^2/2) are computed in
 * double on the host and rounded once to float.  *out receives the handle.
 * Errors: SIM_EINVAL (bad sizes/values, *out untouched), SIM_ENOMEM, SIM_EHIP. */
int sim_create(const sim_network* net, const sim_params* params, void* hip_stream,
               sim_alloc_fn alloc, sim_free_fn free_fn, void* alloc_ctx, sim_t** out);

/* Load the trips (Sec. 6.2.2 departure times, Sec. 6.3.1 routes).  Once per
 * handle.  HOST arrays:
 *   depart_step [num_trips]   step at which the trip becomes due (>= current step)
 *   trip_route  [num_trips]   route id per trip (routes may be shared)
 *   route_ptr   [num_routes+1] offsets into route_edges (int64, total < 2^31)
 *   route_edges [route_ptr[num_routes]]  consecutive edges must be joined
 *   init_x/init_v/init_lane   NULL, or [num_trips] each: every trip is then
 *                             placed on the first edge of its route at that
 *                             position (front bumper, m), speed and lane, all
 *                             with depart_step == current step, no overlap.
 * Vehicle id = rank of the trip by (depart_step, trip index); lower ids win
 * conflicting claims.  All-or-nothing: on error nothing is loaded.
 * Errors: SIM_EINVAL, SIM_EROUTE, SIM_ESTATE (second call, departure in the
 * past), SIM_ENOMEM, SIM_EHIP. */
int sim_load_demand(sim_t* sim, int32_t num_trips, const int32_t* depart_step,
                    const int32_t* trip_route, int32_t num_routes, const int64_t* route_ptr,
                    const int32_t* route_edges, const float* init_x, const float* init_v,
                    const int32_t* init_lane);

/* New routes for the same trips, handed over on the DEVICE, and the demand
 * started again from its first step (Sec. 6.3.1: each iteration of the
 * decaying re-routing simulates the whole horizon again with the re-planned
 * routes).  route_ptr: DEVICE int64 [num_trips + 1], route_ptr[0] = 0,
 * strictly increasing; route i = route_edges[route_ptr[i] .. route_ptr[i+1])
 * (DEVICE int32 [total_route_edges]) is the route of trip i in the order of
 * the sim_load_demand call (the table rt_route_views exposes).  Both arrays
 * are copied; the caller keeps them.  Every route is checked on the device
 * (non-empty, edge ids in range, consecutive edges meeting at a node) before
 * anything changes.  The trips keep their departure steps and types; their
 * departure queues (first link, type) are rebuilt for the new first links;
 * the state goes back to the step the demand was loaded at: no vehicle on the
 * road, empty queues, zero link statistics and samples, no trip outcomes.
 * Launch shape, control and sampler settings stay.  Synchronises.
 * Errors: SIM_ESTATE (no demand; a demand that placed vehicles on the road; a
 * batch of scenarios; inside a differentiation window), SIM_EINVAL (null or
 * negative arrays, route_ptr[num_trips] != total_route_edges), SIM_EROUTE (a
 * bad route: nothing was changed), SIM_ENOMEM, SIM_EHIP. */
int sim_reload_routes(sim_t* sim, const int64_t* route_ptr, const int32_t* route_edges,
                      int64_t total_route_edges);

/* Advance num_steps synchronous steps (Sec. 6.3.2: lane change, car following,
 * position/speed/travel-time update per vehicle per dt).  Asynchronous: only
 * enqueues kernels.  Errors: SIM_ESTATE (no demand), SIM_EINVAL, SIM_EHIP. */
int sim_step(sim_t* sim, int32_t num_steps);

/* Read counters into host_out (synchronises), and enqueue device-to-device
 * copies of the per-edge statistics into the DEVICE arrays edge_count,
 * edge_tt_steps (sum of whole steps spent on the edge) and edge_tt_us (sum of
 * crossing-interpolated traversal times, microseconds), each [num_edges].
 * Every pointer may be NULL. */
int sim_stats(sim_t* sim, sim_stats_t* host_out, int64_t* edge_count, int64_t* edge_tt_steps,
              int64_t* edge_tt_us);

/* Copy the vehicles on the road to HOST arrays of capacity `cap` (in the
 * library's lane order; synchronises).  *n_out = number on the road (if it
 * exceeds cap nothing is copied and SIM_EINVAL is returned).  Any array may
 * be NULL.  cursor = index of the current edge within the vehicle's route;
 * lc = step of the last lane change; kin/phin = entry step / fraction; fuel (mL)
 * and co (g) = accumulated so far (Sec. 6.3.4). */
int sim_read_vehicles(sim_t* sim, int32_t cap, int32_t* n_out, int32_t* vid, int32_t* edge,
                      int32_t* lane, int32_t* cursor, int32_t* lc, int32_t* kin, float* x,
                      float* v, float* phin, float* fuel, float* co);

/* Copy per-vehicle-id outcomes to HOST arrays [num_trips]: the step at which the
 * vehicle appeared on the road (-1 if not yet) and the first step after its
 * arrival (-1 if not arrived).  Synchronises. */
int sim_read_trips(sim_t* sim, int32_t* depart_actual, int32_t* arrive_step);

/* Fuel (mL) and CO (g) of every vehicle id over its whole trip, written at its
 * arrival (0 before), to HOST arrays [num_trips].  Per step each vehicle adds
 * rate*dt: fuel rate 0.666 + 0.072*max(0, 0.269v + 0.0171v^2 + 0.000672v^3 +
 * 1.680av + P_ea), P_ea = 0.79296a^2v for a > 0 (v in m/s, a = realized
 * acceleration of the step); CO rate -0.064 + 0.0056vm + 0.00026(vm-50)^2 (vm in
 * mph) -- the two equations of Sec. 6.3.4.  Synchronises. */
int sim_read_emissions(sim_t* sim, float* fuel, float* co);

/* Utilization / speed sampler (Sec. 6.4): every `every` steps (120 = 1 min at
 * dt = 0.5 s) each link adds its number of vehicles and the sum of their speeds
 * (micrometres per second, rounded) to sample group floor(t/every)/group
 * (group 6 = 6-minute averages); groups beyond max_groups are dropped.
 * Allocates 16 B x max_groups x num_edges of device memory.  Utilization of a
 * link in a group = count / (group * length * lanes / (veh_length + s0)). */
int sim_set_sampler(sim_t* sim, int32_t every, int32_t group, int32_t max_groups);

/* Copy the sampler sums to HOST arrays [max_groups][num_edges].  Synchronises. */
int sim_read_samples(sim_t* sim, int64_t* count, int64_t* speed_um);

/* Replace the IDM parameters (same num_classes) between steps; derived
 * constants are recomputed as in sim_create.  Errors: SIM_EINVAL. */
int sim_set_idm(sim_t* sim, const float* idm);

/* Vehicle types (Sec. 6.3.5: trucks differ from cars in size, acceleration
 * and maximum speed).  types: HOST float [num_types][3] = (length in m,
 * acceleration cap in m/s^2, speed cap in m/s); a cap may be +inf.  A vehicle
 * of type k has length types[k][0] (gaps to it, its claim cells, its entry
 * point x = length); its car-following uses a = min(a_class, cap_a) and
 * v0 = min(v0_scale * speed limit, cap_v).  trip_type: HOST uint8 [num_trips]
 * in the trip order of sim_load_demand (NULL: every trip type 0).  Without
 * this call there is one type: (veh_length, +inf, +inf).  1 <= num_types <= 4;
 * every link must be at least as long as every type plus s0.  Must precede
 * sim_load_demand (for ensembles: the concatenated trips, scenario order).
 * Errors: SIM_EINVAL, SIM_ESTATE (demand already loaded). */
int sim_set_vehicle_types(sim_t* sim, int32_t num_types, const float* types, int32_t num_trips,
                          const uint8_t* trip_type);

/* Intersection control (Sec. 6.3.2, stop signs and traffic signals).
 * node_control: HOST int32[num_nodes] (copied), 0 = uncontrolled, 1 = stop
 * sign, 2 = signal.  A vehicle whose next movement (link e -> link e') is held
 * sees a stopped vehicle with its rear at the end of e (the stop line).
 *   signal: the node's n inbound x m outbound movements get the green in
 *     turn, signal_green_steps steps each; movement (i, j) is green in phase
 *     i*m + j, where i ranks e among the node's inbound links by link id and
 *     j ranks e' among its outbound links (CSR order);
 *   stop sign: every movement is held except for one admitted vehicle.  A
 *     free node admits, at the start of a step, the lowest-id vehicle whose
 *     front is within stop_dist of its line at speed <= stop_speed and which
 *     goes on to another link; the node is free again once that vehicle has
 *     entered its next link.
 * May be called before or after sim_load_demand, outside a differentiation
 * window; every stop node starts free.  Ensemble handles take the
 * concatenation of the member networks' node arrays.
 * Errors: SIM_EINVAL (null, value not in 0..2, signal_green_steps <= 0,
 * stop_dist <= 0, stop_speed < 0), SIM_ESTATE (inside a window), SIM_ENOMEM. */
int sim_set_control(sim_t* sim, const int32_t* node_control, int32_t signal_green_steps, float stop_dist,
                    float stop_speed);

/* Per-kernel timing with HIP events on the handle's stream: when every > 0,
 * every `every`-th subsequent step launches each of its SIM_NUM_KERNELS
 * kernels (decide, resolve, scan, scatter, place, lanes) with a start
 * and a stop event of its own (hipExtLaunchKernelGGL), which take that
 * kernel's begin and end timestamps; 0 disables.  Timing adds no
 * synchronisation to sim_step. */
#define SIM_NUM_KERNELS 6
int sim_set_timing(sim_t* sim, int32_t every);

/* Synchronise, then add the elapsed milliseconds of every sampled launch to
 * kernel_ms[SIM_NUM_KERNELS] (HOST) and store the number of sampled steps in
 * *samples; the sampled events are released. */
int sim_read_timing(sim_t* sim, double* kernel_ms, int64_t* samples);

/* State views, checkpoint and resume.
 *
 * The vehicles on the road at the current step, as DEVICE arrays owned by the
 * handle (valid until the next call that advances or replaces the state),
 * num_vehicles entries each, sorted by (key, x): key = global lane id =
 * lane_base[edge] + lane, where lane_base is the exclusive prefix sum of the
 * lanes of the edges in edge-id order; x = front-bumper position from the link
 * start (m); v = speed (m/s); edge; vid = vehicle id (rank of the trip by
 * (departure step, trip index)); type = vehicle type. */
typedef struct {
    int64_t step;
    int32_t num_vehicles;
    const int32_t* key;
    const float* x;
    const float* v;
    const int32_t* edge;
    const int32_t* vid;
    const uint8_t* type;
} sim_state_view;

/* Size in bytes of a state image of this handle (after sim_load_demand). */
int sim_state_bytes(sim_t* sim, size_t* bytes);

/* Fill *out with the current step, vehicle count and views; if image is not
 * NULL, also copy the whole dynamic state into it: DEVICE memory of
 * sim_state_bytes bytes, owned by the caller (vehicles, departure queues,
 * counters, stop-node holders, per-trip outcomes, emissions and link
 * statistics; not the utilization samples).  Synchronises.
 * Errors: SIM_EINVAL (null out), SIM_ESTATE (no demand), SIM_EHIP. */
int sim_get_state(sim_t* sim, sim_state_view* out, void* image);

/* Replace the dynamic state by an image (DEVICE, `bytes` bytes) written by
 * sim_get_state of this handle or of another one created with the same
 * network, parameters, vehicle types and demand; the simulation continues from
 * the image's step exactly as the one that wrote it would.  The image is
 * validated first, on the device, against every class of sim_check_state; an
 * image that fails is refused with nothing copied (sim_last_error names the
 * first failing class, its count and its lowest entry).  Synchronises.
 * Errors: SIM_EINVAL (null, wrong size, an image of a different simulation,
 * or one that fails validation), SIM_ESTATE (no demand, or inside a
 * differentiation window), SIM_ENOMEM, SIM_EHIP. */
int sim_set_state(sim_t* sim, const void* image, size_t bytes);

/* Classes of violations that sim_check_state counts: what the step kernels
 * assume of a state, since they index link, lane, route, trip and queue
 * arrays with its values and take the vehicles of a lane as consecutive
 * entries ordered by position (Sec. 6.3.3, the per-lane order of vehicles). */
enum sim_check_class {
    SIM_CHECK_COUNT = 0, /* vehicle count outside [0, capacity], or a negative step */
    SIM_CHECK_KEY,       /* lane key outside [0, total lanes) */
    SIM_CHECK_EDGE,      /* link out of range, or the lane key not one of its lanes */
    SIM_CHECK_ORDER,     /* entries not ordered by (lane key, position) */
    SIM_CHECK_POSITION,  /* position not finite, or negative */
    SIM_CHECK_SPEED,     /* speed not finite, or negative */
    SIM_CHECK_VID,       /* vehicle id outside [0, trips) */
    SIM_CHECK_DUPLICATE, /* a vehicle id on the road twice */
    SIM_CHECK_TYPE,      /* vehicle type out of range, or not its trip's type */
    SIM_CHECK_ROUTE,     /* route cursor outside the trip's route, or the route's link there not the vehicle's */
    SIM_CHECK_NEXT,      /* next link not the route's next one (-1 after the last) */
    SIM_CHECK_VALUE,     /* link-entry fraction outside [0, 1], or fuel or CO not finite */
    SIM_CHECK_ARRIVED,   /* a vehicle on the road whose trip already has an arrival step */
    SIM_CHECK_QUEUE,     /* a departure queue's head past its tail, or its tail past its trips */
    SIM_CHECK_HOLDER,    /* a stop node's holder neither -1 nor a vehicle id */
    SIM_CHECK_CLASSES
};

/* Check the current state against every class above (one device pass over
 * the vehicles on the road, the departure queues and the stop nodes; each
 * index is tested before it is used).
 *   counts [SIM_CHECK_CLASSES]  HOST int64 out: violations per class (all 0: valid)
 *   first  [SIM_CHECK_CLASSES]  HOST int32 out, may be NULL: lowest offending
 *                               entry (sorted position, queue or node) per
 *                               class, INT32_MAX where there is none
 * A state the step itself produced passes.  Synchronises.  Errors: SIM_EINVAL
 * (null counts), SIM_ESTATE (no demand), SIM_ENOMEM, SIM_EHIP. */
int sim_check_state(sim_t* sim, int64_t* counts, int32_t* first);

/* Start a differentiation window at the current step: subsequent sim_step
 * calls save a full-state checkpoint every `checkpoint_every` steps (device
 * memory, ~44 B x trips each).  At most 16 link classes.  Errors: SIM_EINVAL,
 * SIM_ESTATE (no demand). */
int sim_tape_begin(sim_t* sim, int32_t checkpoint_every);

/* Gradient of a loss of the per-link mean travel times (Sec. 6.4) with respect
 * to the IDM parameters (Sec. 6.3.2, car-following equation) of every link
 * class, over the window since sim_tape_begin, with every discrete event of
 * that window (who is on which link and lane, who follows whom, when a link
 * end is crossed, which branch each min/max/stop/clamp took) held fixed.
 *   dL_dmeanTT [num_edges]        DEVICE float: dLoss/d(mean travel time of the
 *                                 link in seconds), mean = tt_us / count / 1e6
 *   dL_dtheta  [num_classes * 4]  DEVICE float out: (v0_scale, T, a, b) per class
 * Each checkpointed segment is recomputed with its event tape, then walked
 * backwards.  Asynchronous on the handle's stream; live state and statistics
 * are left as they were.  Errors: SIM_ESTATE (no window), SIM_ENOMEM, SIM_EHIP. */
int sim_grad(sim_t* sim, const float* dL_dmeanTT, float* dL_dtheta);

/* Frozen-event replay of the differentiation window at other IDM parameters,
 * for finite-difference checks of sim_grad at the same accuracy: every
 * vehicle moves exactly as recorded (who follows whom, lanes, links, crossing
 * steps, the branch of every min/max/stop/clamp), only positions and speeds
 * are recomputed, from the recorded state at the window start, with
 *   idm [num_classes * 4]  HOST double: (v0_scale, T, a, b) per class
 * in the step's own expressions: in float (fp64 = 0; the parameters rounded
 * to float, the constants computed as the simulator's), where at the recorded
 * parameters the replay reproduces the recorded trajectory bit for bit, or in
 * double throughout (fp64 != 0), from the recorded float state.  With every
 * branch held, a parameter far from the recorded one can make a held branch
 * meaningless (a gap forced positive that closes, a stop with a positive
 * acceleration), and the replay then yields non-finite sums; differences of
 * about 1e-6 stay clear of that.  Writes, per link, the sum
 * over the window's completed traversals of (exit fraction - entry fraction):
 *   frac_sum [num_edges]   HOST double
 * so the mean travel time at idm is the recorded one plus
 * dt * (frac_sum(idm) - frac_sum(recorded)) / count.  Needs a window recorded
 * as one segment (sim_tape_begin with a checkpoint interval at least its
 * length); the first replay (or sim_grad) recomputes the window from its
 * checkpoint with the event tape on, later replays reuse that tape.
 * Synchronises; the live parameters and state are left as they were.
 * Errors: SIM_EINVAL (parameters out of range), SIM_ESTATE, SIM_ENOMEM, SIM_EHIP. */
int sim_replay(sim_t* sim, const double* idm, int32_t fp64, double* frac_sum);

/* Batched ensemble: n scenarios simulated as one (their networks side by side:
 * node, edge, lane and class ids of scenario q are offset by the totals of
 * scenarios 0..q-1).  Every field of params[q] except idm/num_classes must
 * equal params[0].  Vehicles of different scenarios never share a lane, and a
 * trip's vehicle id keeps its scenario's (departure, index) order, so every
 * scenario evolves exactly as in its own simulation.  Errors as sim_create. */
int sim_create_batch(int32_t n, const sim_network* nets, const sim_params* params, void* hip_stream,
                     sim_alloc_fn alloc, sim_free_fn free_fn, void* alloc_ctx, sim_t** out);

/* Demand of a batch: for each scenario q the arrays of sim_load_demand (HOST,
 * edge ids local to scenario q); placed trips are not supported here.  Trips
 * are concatenated in scenario order.  Errors as sim_load_demand. */
int sim_load_demand_batch(sim_t* sim, int32_t n, const int32_t* num_trips, const int32_t* const* depart_step,
                          const int32_t* const* trip_route, const int32_t* num_routes,
                          const int64_t* const* route_ptr, const int32_t* const* route_edges);

/* Launch shape: blocks for the per-vehicle, per-claim and per-mover kernels
 * (grid; 256 threads each except the decide kernel, see below) and for the
 * persistent blocks of the step's scan (grid_small).  Results do not depend
 * on the shape. */
int sim_set_launch(sim_t* sim, int32_t grid, int32_t grid_small);
int sim_get_launch(sim_t* sim, int32_t* grid, int32_t* grid_small);

/* The decide kernel's shape: threads per block and sorted vehicle entries per
 * thread (a block takes tiles of block x per_thread entries, staged in LDS).
 * Supported: (256, 1) the default, (256, 2), (128, 1), (128, 2), (512, 1),
 * (256, 4).  Results do not depend on the shape.  Errors: SIM_EINVAL (not
 * supported), SIM_ESTATE (after the adjoint buffers were sized). */
int sim_set_decide_shape(sim_t* sim, int32_t block, int32_t per_thread);
int sim_get_decide_shape(sim_t* sim, int32_t* block, int32_t* per_thread);

/* As sim_step, with runs of `chunk` consecutive steps replayed from captured
 * HIP graphs (captured on first use per run length and step parity).  With
 * timing on (sim_set_timing), each sampled step runs alone and the runs stop
 * at it.  Falls back to sim_step while a differentiation window is active. */
int sim_step_graph(sim_t* sim, int32_t num_steps, int32_t chunk);

/* The same steps as sim_step in one persistent launch (up to 600 steps per
 * launch): the device's resident blocks (a cooperative launch) take the
 * step's phases in turn with a device-wide barrier between phases, each phase
 * over the virtual grid of its own launch, so results are identical to
 * sim_step.  Needs a decide shape of 256 threads and 1 or 2 entries per
 * thread.  With a differentiation window or per-kernel timing active, falls
 * back to sim_step.  Synchronises at the end and checks the barriers: a
 * barrier that gave up waiting (the launch could not keep every block
 * resident) makes the call fail with SIM_EHIP, and the state is then void.
 * Errors: SIM_EINVAL, SIM_ESTATE, SIM_ENOMEM, SIM_EHIP. */
int sim_step_persistent(sim_t* sim, int32_t num_steps);

/* Time `steps_per_trial` steps for each candidate launch shape, all from the
 * current state (every candidate twice): grid counts with the scan's blocks a
 * share of them (1/2, 1/4, 1/8) or 128 or 256, then every decide shape with
 * the best grid, half and twice it.  Then
 * restore that state (vehicles, counters, statistics, per-trip outcomes, the
 * sampler setting) and keep the fastest shape (read the decide shape with
 * sim_get_decide_shape).  Outputs the grids and the time per step (ms).  The
 * copy of the state it allocates is freed before it returns; on an error the
 * state is restored as far as possible and some shape is kept.
 * Synchronises. */
int sim_autotune(sim_t* sim, int32_t steps_per_trial, int32_t* best_grid, int32_t* best_small, float* best_ms);

/* Route subsequent work to another HIP stream. */
int sim_set_stream(sim_t* sim, void* hip_stream);

/* Free all device memory of the handle (synchronises its stream). */
void sim_destroy(sim_t* sim);

/* Text of the last error on this handle ("" if none); valid until the next
 * call on the handle.  sim_strerror: fixed text of a SIM_E* code. */
const char* sim_last_error(const sim_t* sim);
const char* sim_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* TRAFFICSIM_H */
