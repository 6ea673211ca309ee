/*
 * CPU ORACLE for the traffic microsimulation step -- test infrastructure only.
 *
 * Plain, slow, obviously-correct C.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the product library never
 * does.  It shares no code, header, table or constant generator with the HIP
 * path.  The same source is compiled twice: -DORACLE_F64 gives the FP64
 * oracle, without it the FP32 oracle.  Build flags: -O2 -ffp-contract=off
 * -fno-fast-math (no FMA contraction, IEEE round-to-nearest-even).
 *
 * What it computes (one synchronous step t -> t+1; every decision reads
 * state t only):
 *   - car following: the Intelligent Driver Model of Sec. 6.3.2
 *     (the car-following equation, exponent 4, v0 = desired speed of the
 *     link, s = gap to the vehicle ahead);
 *   - lane changes, mandatory or discretionary, each subject to gap
 *     acceptance (Sec. 6.3.2, lane-changing and gap-acceptance items);
 *   - route traversal: every vehicle follows its precomputed edge list from
 *     origin to destination (Sec. 6.2.1, Sec. 6.3.1) with time step dt
 *     (Sec. 6.3.2, dt = 0.5 s);
 *   - departures from per-trip departure steps (Sec. 6.2.2);
 *   - per-link traversal statistics (Sec. 6.4).
 * Where the paper is silent the readings are the documented ones: ballistic
 * integration, MOBIL incentive for discretionary changes, a distance
 * threshold for the mandatory state, one-metre claim cells with the
 * lowest-vehicle-id-wins rule for merges, lane changes and insertions.
 *
 * Parity: pinned by closed forms (free-road acceleration from rest, ring-road
 * equilibrium), invariants (conservation, no overlap within a lane) and an
 * independent brute-force implementation on tiny networks.  The lane-choice
 * and intersection behaviour beyond those invariants is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_F64
typedef double real;
#define RFLOOR floor
#define RRINT rint
#else
typedef float real;
#define RFLOOR floorf
#define RRINT rintf
#endif

#define RMAX(a, b) ((a) > (b) ? (a) : (b))
#define RMIN(a, b) ((a) < (b) ? (a) : (b))
#define LC_NONE (-(1 << 30))

enum { OR_OK = 0, OR_EINVAL = -1, OR_EROUTE = -2, OR_ENOMEM = -3, OR_ESTATE = -5 };
enum { K_STAY = 0, K_ARRIVE = 1, K_CROSS = 2, K_CHANGE = 3 };
/* modes of the event tape */
enum { TM_STAY = 0, TM_CHANGE = 1, TM_YIELD = 2, TM_ARRIVE = 3, TM_CROSS = 4, TM_APPEAR = 5 };

typedef struct {
    int32_t vid, edge, lane, rcur, next, lc, kin;
    int32_t ty; /* vehicle type (0 car; Sec. 6.3.5 adds trucks) */
    real x, v, phin;
    real fuel, co; /* accumulated fuel (mL) and CO (g) */
} veh_t;

typedef struct {
    /* network */
    int32_t nn, ne, nlanes;
    /* intersection control per node: 0 none, 1 stop, 2 signal (Sec. 6.3.2) */
    int32_t *ctrl, *holder, *in_rank, *in_deg;
    int32_t green;
    real stop_dist, stop_speed;
    int32_t *row_ptr, *col_idx, *lanes, *cls, *lane_base, *ncell;
    real *len, *inv_v0; /* inv_v0[e * nt + type] */
    /* parameters */
    int32_t ncls, lc_cool;
    real dt, h, lveh, s0, claim_len, s_eps, b_max, p, athr, bsafe, dmand, dt_us_f;
    int64_t dt_us;
    real *T, *A, *kab; /* A, kab: [class * nt + type] */
    /* vehicle types (Sec. 6.3.5): length, acceleration cap, speed cap */
    int32_t nt;
    real tlen[4], tclaim[4];
    double tamax[4], tvmax[4];
    float *idm_in, *speed_in; /* inputs the per-type constants are derived from */
    uint8_t* trip_type; /* per trip (input order), set before loading */
    int32_t ntyped;
    int32_t* vtype;     /* per vehicle id */
    real mph; /* miles per hour per m/s */
    /* demand, indexed by vehicle id */
    int32_t ntrips, loaded;
    int32_t *dep, *rbeg, *rend, *route_edges;
    int64_t nroute_edges;
    int32_t *depart_actual, *arrive_step;
    /* state */
    int32_t t, nact, npend, relc;
    veh_t* act;
    int32_t* pend;
    int64_t *st_cnt, *st_steps, *st_us;
    int64_t departed, arrived, updates, claims_lost, clamps;
    int64_t claims, claims_dep, lc_evaluated, claims_lc;
    real *fuel_total, *co_total; /* per vehicle id, at arrival */
    /* sampler: every `samp_every` steps, per link vehicle count and speed sum
     * (micrometres per second), accumulated in groups of `samp_group` samples */
    int32_t samp_every, samp_group, samp_max;
    int64_t *samp_cnt, *samp_spd;
    /* event tape (discrete outcomes of every step, for the frozen-event replay) */
    int tape_on;
    int64_t tp_n, tp_cap;
    int32_t *tp_step, *tp_vid, *tp_mode, *tp_lead, *tp_flags, *tp_edge;
    double *tp_x0, *tp_v0;
} osim;

static void tape_push(osim* S, int32_t step, int32_t vid, int32_t mode, int32_t lead, int32_t flags,
                      int32_t edge, double x0, double v0) {
    if (!S->tape_on) return;
    if (S->tp_n == S->tp_cap) {
        int64_t c = S->tp_cap ? 2 * S->tp_cap : 4096;
        S->tp_step = (int32_t*)realloc(S->tp_step, sizeof(int32_t) * c);
        S->tp_vid = (int32_t*)realloc(S->tp_vid, sizeof(int32_t) * c);
        S->tp_mode = (int32_t*)realloc(S->tp_mode, sizeof(int32_t) * c);
        S->tp_lead = (int32_t*)realloc(S->tp_lead, sizeof(int32_t) * c);
        S->tp_flags = (int32_t*)realloc(S->tp_flags, sizeof(int32_t) * c);
        S->tp_edge = (int32_t*)realloc(S->tp_edge, sizeof(int32_t) * c);
        S->tp_x0 = (double*)realloc(S->tp_x0, sizeof(double) * c);
        S->tp_v0 = (double*)realloc(S->tp_v0, sizeof(double) * c);
        S->tp_cap = c;
    }
    int64_t i = S->tp_n++;
    S->tp_step[i] = step; S->tp_vid[i] = vid; S->tp_mode[i] = mode; S->tp_lead[i] = lead;
    S->tp_flags[i] = flags; S->tp_edge[i] = edge; S->tp_x0[i] = x0; S->tp_v0[i] = v0;
}

/* ------------------------------------------------------------------------ */
/* Per (class, type) and (link, type) car-following constants: a type caps the
 * class's maximum acceleration and the link's desired speed (Sec. 6.3.5:
 * trucks differ in size, acceleration and maximum speed).  In double, rounded
 * once; with no cap (infinite) they are the class's own values. */
static void derive_type_constants(osim* S) {
    const int nt = S->nt;
    free(S->A); free(S->kab); free(S->inv_v0);
    S->A = (real*)malloc(sizeof(real) * S->ncls * nt);
    S->kab = (real*)malloc(sizeof(real) * S->ncls * nt);
    S->inv_v0 = (real*)malloc(sizeof(real) * S->ne * nt);
    for (int c = 0; c < S->ncls; ++c) {
        double a = S->idm_in[4 * c + 2], b = S->idm_in[4 * c + 3];
        S->T[c] = (real)S->idm_in[4 * c + 1];
        for (int k = 0; k < nt; ++k) {
            double ak = a < S->tamax[k] ? a : S->tamax[k];
            S->A[c * nt + k] = (real)ak;
            S->kab[c * nt + k] = (real)(1.0 / (2.0 * sqrt(ak * b)));
        }
    }
    for (int32_t e = 0; e < S->ne; ++e) {
        double v0 = (double)S->idm_in[4 * S->cls[e] + 0] * (double)S->speed_in[e];
        for (int k = 0; k < nt; ++k) S->inv_v0[e * nt + k] = (real)(1.0 / (v0 < S->tvmax[k] ? v0 : S->tvmax[k]));
    }
}

/* Vehicle types (Sec. 6.3.5), before or_load_demand: types[nt][3] = (length,
 * acceleration cap, speed cap; caps may be +inf), trip_type[ntrips] in input
 * order (NULL: all type 0).  Every link must hold the longest type. */
int or_set_vehicle_types(osim* S, int32_t nt, const float* types, int32_t ntrips, const uint8_t* trip_type) {
    if (S->loaded) return OR_ESTATE;
    if (nt < 1 || nt > 4 || ntrips < 0) return OR_EINVAL;
    for (int k = 0; k < nt; ++k) {
        if (!(types[3 * k] > 0) || !(types[3 * k + 1] > 0) || !(types[3 * k + 2] > 0)) return OR_EINVAL;
        for (int32_t e = 0; e < S->ne; ++e)
            if (!((double)S->len[e] >= (double)types[3 * k] + (double)S->s0)) return OR_EINVAL;
    }
    for (int32_t i = 0; i < ntrips; ++i)
        if (trip_type && trip_type[i] >= nt) return OR_EINVAL;
    S->nt = nt;
    for (int k = 0; k < nt; ++k) {
        S->tlen[k] = (real)types[3 * k];
        S->tclaim[k] = (real)((double)types[3 * k] + (double)S->s0);
        S->tamax[k] = (double)types[3 * k + 1];
        S->tvmax[k] = (double)types[3 * k + 2];
    }
    free(S->trip_type);
    S->trip_type = NULL;
    S->ntyped = ntrips;
    if (trip_type) {
        S->trip_type = (uint8_t*)malloc(ntrips + 1);
        memcpy(S->trip_type, trip_type, ntrips);
    }
    derive_type_constants(S);
    return OR_OK;
}

/* creation: derived constants are computed once in double from the inputs
 * and rounded once to `real`. */
osim* or_create(int32_t nn, int32_t ne, const int32_t* row_ptr, const int32_t* col_idx,
                const int32_t* lanes, const float* length, const float* speed,
                const int32_t* link_class, int32_t ncls, const float* idm,
                const float* fp, int32_t lc_cool, int32_t* err) {
    *err = OR_EINVAL;
    if (nn <= 0 || ne <= 0 || ncls <= 0) return NULL;
    if (row_ptr[0] != 0 || row_ptr[nn] != ne) return NULL;
    osim* S = (osim*)calloc(1, sizeof(osim));
    S->nn = nn; S->ne = ne; S->ncls = ncls; S->lc_cool = lc_cool;
    S->row_ptr = (int32_t*)malloc(sizeof(int32_t) * (nn + 1));
    memcpy(S->row_ptr, row_ptr, sizeof(int32_t) * (nn + 1));
    S->col_idx = (int32_t*)malloc(sizeof(int32_t) * ne);
    S->lanes = (int32_t*)malloc(sizeof(int32_t) * ne);
    S->cls = (int32_t*)malloc(sizeof(int32_t) * ne);
    S->lane_base = (int32_t*)malloc(sizeof(int32_t) * (ne + 1));
    S->ncell = (int32_t*)malloc(sizeof(int32_t) * ne);
    S->len = (real*)malloc(sizeof(real) * ne);
    S->inv_v0 = (real*)malloc(sizeof(real) * ne);
    S->T = (real*)malloc(sizeof(real) * ncls);
    S->A = (real*)malloc(sizeof(real) * ncls);
    S->kab = (real*)malloc(sizeof(real) * ncls);
    S->dt = (real)fp[0];
    S->lveh = (real)fp[1];
    S->s0 = (real)fp[2];
    S->s_eps = (real)fp[3];
    S->b_max = (real)fp[4];
    S->p = (real)fp[5];
    S->athr = (real)fp[6];
    S->bsafe = (real)fp[7];
    S->dmand = (real)fp[8];
    S->h = (real)(0.5 * (double)fp[0] * (double)fp[0]);
    S->claim_len = (real)((double)fp[1] + (double)fp[2]);
    S->dt_us = llround((double)fp[0] * 1e6);
    S->dt_us_f = (real)((double)fp[0] * 1e6);
    S->mph = (real)(1.0 / 0.44704);
    S->nt = 1;
    S->tamax[0] = INFINITY;
    S->tvmax[0] = INFINITY;
    S->tlen[0] = S->lveh;
    S->tclaim[0] = S->claim_len;
    S->idm_in = (float*)malloc(sizeof(float) * 4 * ncls);
    S->speed_in = (float*)malloc(sizeof(float) * ne);
    memcpy(S->idm_in, idm, sizeof(float) * 4 * ncls);
    memcpy(S->speed_in, speed, sizeof(float) * ne);
    for (int c = 0; c < ncls; ++c) {
        double a = idm[4 * c + 2], b = idm[4 * c + 3];
        if (!(a > 0) || !(b > 0) || !(idm[4 * c + 0] > 0) || !(idm[4 * c + 1] >= 0)) goto bad;
    }
    S->lane_base[0] = 0;
    for (int32_t e = 0; e < ne; ++e) {
        int32_t c = link_class ? link_class[e] : 0;
        if (c < 0 || c >= ncls || lanes[e] < 1 || lanes[e] > 8 || !(speed[e] > 0) ||
            !(length[e] >= fp[1] + fp[2]) || col_idx[e] < 0 || col_idx[e] >= nn)
            goto bad;
        S->col_idx[e] = col_idx[e];
        S->lanes[e] = lanes[e];
        S->cls[e] = c;
        S->len[e] = (real)length[e];
        S->ncell[e] = (int32_t)floor((double)length[e]) + 1;
        S->lane_base[e + 1] = S->lane_base[e] + lanes[e];
    }
    S->nlanes = S->lane_base[ne];
    derive_type_constants(S);
    *err = OR_OK;
    return S;
bad:
    *err = OR_EINVAL;
    free(S->row_ptr); free(S->col_idx); free(S->lanes); free(S->cls); free(S->lane_base);
    free(S->ncell); free(S->len); free(S->inv_v0); free(S->T); free(S->A); free(S->kab);
    free(S->idm_in); free(S->speed_in); free(S);
    return NULL;
}

/* Intersection control (Sec. 6.3.2): ctrl[node] = 0 none, 1 stop, 2 signal;
 * a signal cycles through its n_in * m_out movements, `green` steps each; a
 * stop admits one vehicle at a time, chosen among vehicles stopped (speed <=
 * stop_speed) within stop_dist of the line. */
int or_set_control(osim* S, const int32_t* ctrl, int32_t green, float stop_dist, float stop_speed) {
    if (green <= 0 || !(stop_dist > 0) || !(stop_speed >= 0)) return OR_EINVAL;
    if (!S->ctrl) {
        S->ctrl = (int32_t*)calloc(S->nn + 1, sizeof(int32_t));
        S->holder = (int32_t*)malloc(sizeof(int32_t) * (S->nn + 1));
        S->in_rank = (int32_t*)malloc(sizeof(int32_t) * (S->ne + 1));
        S->in_deg = (int32_t*)calloc(S->nn + 1, sizeof(int32_t));
        for (int32_t e = 0; e < S->ne; ++e) S->in_rank[e] = S->in_deg[S->col_idx[e]]++;
    }
    for (int32_t u = 0; u < S->nn; ++u) {
        if (ctrl[u] < 0 || ctrl[u] > 2) return OR_EINVAL;
        S->ctrl[u] = ctrl[u];
        S->holder[u] = -1;
    }
    S->green = green;
    S->stop_dist = (real)stop_dist;
    S->stop_speed = (real)stop_speed;
    return OR_OK;
}

void or_destroy(osim* S) {
    if (!S) return;
    free(S->ctrl); free(S->holder); free(S->in_rank); free(S->in_deg);
    free(S->row_ptr); free(S->col_idx); free(S->lanes); free(S->cls); free(S->lane_base);
    free(S->ncell); free(S->len); free(S->inv_v0); free(S->T); free(S->A); free(S->kab);
    free(S->idm_in); free(S->speed_in); free(S->trip_type); free(S->vtype);
    free(S->dep); free(S->rbeg); free(S->rend); free(S->route_edges);
    free(S->depart_actual); free(S->arrive_step); free(S->act); free(S->pend);
    free(S->st_cnt); free(S->st_steps); free(S->st_us);
    free(S->tp_step); free(S->tp_vid); free(S->tp_mode); free(S->tp_lead); free(S->tp_flags);
    free(S->tp_edge); free(S->tp_x0); free(S->tp_v0);
    free(S->fuel_total); free(S->co_total); free(S->samp_cnt); free(S->samp_spd);
    free(S);
}

/* ------------------------------------------------------------------------ */
/* demand: vehicle id = rank of the trip by (departure step, trip index).   */
static const int32_t* g_sort_dep;
static int cmp_trip(const void* a, const void* b) {
    int32_t i = *(const int32_t*)a, j = *(const int32_t*)b;
    if (g_sort_dep[i] != g_sort_dep[j]) return g_sort_dep[i] < g_sort_dep[j] ? -1 : 1;
    return (i > j) - (i < j);
}

static int32_t tail_of(const osim* S, int32_t e) {
    int32_t lo = 0, hi = S->nn; /* largest node u with row_ptr[u] <= e */
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) / 2;
        if (S->row_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

static int32_t lane_key(const osim* S, int32_t e, int32_t l) { return S->lane_base[e] + l; }

/* order used for lanes: (lane key, x, vehicle id) */
static const osim* g_S;
static const veh_t* g_act;
static int cmp_order(const void* a, const void* b) {
    const veh_t* u = &g_act[*(const int32_t*)a];
    const veh_t* w = &g_act[*(const int32_t*)b];
    int32_t ku = lane_key(g_S, u->edge, u->lane), kw = lane_key(g_S, w->edge, w->lane);
    if (ku != kw) return ku < kw ? -1 : 1;
    if (u->x != w->x) return u->x < w->x ? -1 : 1;
    return (u->vid > w->vid) - (u->vid < w->vid);
}

int or_load_demand(osim* S, int32_t ntrips, const int32_t* depart_step, const int32_t* trip_route,
                   int32_t nroutes, const int64_t* route_ptr, const int32_t* route_edges,
                   const float* init_x, const float* init_v, const int32_t* init_lane) {
    if (S->loaded) return OR_ESTATE;
    if (ntrips < 0 || nroutes < 0 || (ntrips > 0 && nroutes == 0)) return OR_EINVAL;
    if (route_ptr[0] != 0) return OR_EROUTE;
    int64_t nre = route_ptr[nroutes];
    if (nre < 0 || nre > INT32_MAX - 2) return OR_EROUTE;
    int32_t* tail = (int32_t*)malloc(sizeof(int32_t) * (S->ne + 1));
    for (int32_t e = 0; e < S->ne; ++e) tail[e] = tail_of(S, e);
    for (int32_t r = 0; r < nroutes; ++r) {
        int bad = route_ptr[r + 1] <= route_ptr[r];
        for (int64_t k = route_ptr[r]; k < route_ptr[r + 1] && !bad; ++k) {
            int32_t e = route_edges[k];
            if (e < 0 || e >= S->ne) bad = 1;
            else if (k + 1 < route_ptr[r + 1] && (route_edges[k + 1] < 0 || route_edges[k + 1] >= S->ne ||
                                                  S->col_idx[e] != tail[route_edges[k + 1]]))
                bad = 1;
        }
        if (bad) {
            free(tail);
            return OR_EROUTE;
        }
    }
    free(tail);
    for (int32_t i = 0; i < ntrips; ++i) {
        if (trip_route[i] < 0 || trip_route[i] >= nroutes) return OR_EINVAL;
        if (depart_step[i] < S->t) return OR_ESTATE;
        if (init_x && depart_step[i] != S->t) return OR_EINVAL;
    }
    int32_t* ord = (int32_t*)malloc(sizeof(int32_t) * (ntrips + 1));
    for (int32_t i = 0; i < ntrips; ++i) ord[i] = i;
    g_sort_dep = depart_step;
    qsort(ord, ntrips, sizeof(int32_t), cmp_trip);
    S->ntrips = ntrips;
    S->dep = (int32_t*)malloc(sizeof(int32_t) * (ntrips + 1));
    S->rbeg = (int32_t*)malloc(sizeof(int32_t) * (ntrips + 1));
    S->rend = (int32_t*)malloc(sizeof(int32_t) * (ntrips + 1));
    S->depart_actual = (int32_t*)malloc(sizeof(int32_t) * (ntrips + 1));
    S->arrive_step = (int32_t*)malloc(sizeof(int32_t) * (ntrips + 1));
    S->fuel_total = (real*)calloc(ntrips + 1, sizeof(real));
    S->co_total = (real*)calloc(ntrips + 1, sizeof(real));
    S->nroute_edges = nre;
    S->route_edges = (int32_t*)malloc(sizeof(int32_t) * (nre + 1));
    memcpy(S->route_edges, route_edges, sizeof(int32_t) * nre);
    if (S->trip_type && S->ntyped != ntrips) {
        free(ord);
        return OR_EINVAL;
    }
    S->vtype = (int32_t*)malloc(sizeof(int32_t) * (ntrips + 1));
    for (int32_t v = 0; v < ntrips; ++v) {
        int32_t i = ord[v];
        S->vtype[v] = S->trip_type ? (int32_t)S->trip_type[i] : 0;
        S->dep[v] = depart_step[i];
        S->rbeg[v] = (int32_t)route_ptr[trip_route[i]];
        S->rend[v] = (int32_t)route_ptr[trip_route[i] + 1];
        S->depart_actual[v] = -1;
        S->arrive_step[v] = -1;
    }
    S->act = (veh_t*)malloc(sizeof(veh_t) * (ntrips + 1));
    S->pend = (int32_t*)malloc(sizeof(int32_t) * (ntrips + 1));
    S->st_cnt = (int64_t*)calloc(S->ne, sizeof(int64_t));
    S->st_steps = (int64_t*)calloc(S->ne, sizeof(int64_t));
    S->st_us = (int64_t*)calloc(S->ne, sizeof(int64_t));
    S->nact = 0;
    S->npend = 0;
    if (init_x) {
        /* placed vehicles enter state t directly, without a claim */
        for (int32_t v = 0; v < ntrips; ++v) {
            int32_t i = ord[v];
            veh_t* q = &S->act[v];
            q->vid = v;
            q->ty = S->vtype[v];
            q->rcur = S->rbeg[v];
            q->edge = S->route_edges[q->rcur];
            q->next = (q->rcur + 1 < S->rend[v]) ? S->route_edges[q->rcur + 1] : -1;
            q->lane = init_lane ? init_lane[i] : 0;
            q->x = (real)init_x[i];
            q->v = init_v ? (real)init_v[i] : (real)0;
            q->lc = LC_NONE;
            q->kin = S->t;
            q->phin = (real)1;
            q->fuel = (real)0;
            q->co = (real)0;
            if (q->lane < 0 || q->lane >= S->lanes[q->edge] || !(init_x[i] >= 0) ||
                !(init_x[i] <= (float)S->len[q->edge]) || (init_v && !(init_v[i] >= 0))) {
                free(ord);
                return OR_EINVAL;
            }
        }
        S->nact = ntrips;
        /* no overlap within a lane */
        int32_t* o = (int32_t*)malloc(sizeof(int32_t) * (ntrips + 1));
        for (int32_t k = 0; k < ntrips; ++k) o[k] = k;
        g_S = S; g_act = S->act;
        qsort(o, ntrips, sizeof(int32_t), cmp_order);
        for (int32_t k = 0; k + 1 < ntrips; ++k) {
            const veh_t *a = &S->act[o[k]], *b = &S->act[o[k + 1]];
            if (a->edge == b->edge && a->lane == b->lane && ((b->x - S->tlen[b->ty]) - a->x) < 0) {
                free(o); free(ord);
                S->nact = 0;
                return OR_EINVAL;
            }
        }
        free(o);
        for (int32_t v = 0; v < ntrips; ++v) {
            S->depart_actual[v] = S->t;
            tape_push(S, S->t, v, TM_APPEAR, -1, 0, S->act[v].edge, (double)S->act[v].x, (double)S->act[v].v);
        }
        S->departed = ntrips;
    }
    free(ord);
    S->loaded = 1;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* the car-following law and the kinematic update                             */
typedef struct {
    int kind;   /* 0 free road, 1 same link, 2 first vehicle of the next link, 3 stop line */
    real s;     /* bumper-to-bumper gap (m) */
    real vl;    /* speed of the vehicle ahead */
    real xl;    /* its front position on its own link */
    int32_t vid;
    real ll;    /* its length */
} lead_t;

/* branch flags of one applied motion (recorded in the event tape) */
enum {
    TF_HAS_LEAD = 1, TF_LEAD_CROSS = 2, TF_DYN_FLOOR = 4, TF_S_FLOOR = 8, TF_ACC_FLOOR = 16,
    TF_STOP = 32, TF_DX_FLOOR = 64, TF_CLAMP = 128, TF_CLAMP_ZERO = 256, TF_CLAMP_V = 512, TF_F_ONE = 1024,
    TF_VIRTUAL = 2048
};
static int lead_flags(lead_t L) {
    if (L.kind == 0) return 0;
    return TF_HAS_LEAD | (L.kind == 2 ? TF_LEAD_CROSS : 0) | (L.kind == 3 ? TF_VIRTUAL : 0);
}

/* IDM acceleration (Sec. 6.3.2, car-following equation), with the dynamic
 * part of the desired gap floored at 0, the gap floored at s_eps and the
 * result floored at -b_max. */
static real idm_fl(const osim* S, int32_t c, int32_t ty, real inv_v0, real v, lead_t L, int* fl) {
    const real A = S->A[c * S->nt + ty], kab = S->kab[c * S->nt + ty];
    real r = v * inv_v0;
    real r2 = r * r;
    real r4 = r2 * r2;
    real fr = (real)1 - r4;
    real acc;
    int f = 0;
    if (L.kind == 0) {
        acc = A * fr;
    } else {
        real dv = v - L.vl;
        real dyn = v * S->T[c] + (v * dv) * kab;
        if ((real)0 > dyn) f |= TF_DYN_FLOOR;
        real ss = S->s0 + RMAX((real)0, dyn);
        if (!(L.s > S->s_eps)) f |= TF_S_FLOOR;
        real q = ss / RMAX(L.s, S->s_eps);
        acc = A * (fr - q * q);
    }
    if (!(acc > -S->b_max)) f |= TF_ACC_FLOOR;
    if (fl) *fl |= f;
    return RMAX(acc, -S->b_max);
}

static real idm(const osim* S, int32_t c, int32_t ty, real inv_v0, real v, lead_t L) {
    return idm_fl(S, c, ty, inv_v0, v, L, NULL);
}

/* Ballistic update over dt; when the speed would turn negative the vehicle
 * stops within the step. */
static void move_fl(const osim* S, real v, real acc, real* dx, real* vn, int* fl) {
    real vv = v + acc * S->dt;
    int f = 0;
    if (vv < (real)0) {
        *dx = (v * v) / ((real)(-2) * acc);
        *vn = (real)0;
        f |= TF_STOP;
    } else {
        *dx = v * S->dt + acc * S->h;
        *vn = vv;
    }
    if (!(*dx > (real)0)) f |= TF_DX_FLOOR;
    *dx = RMAX(*dx, (real)0);
    if (fl) *fl |= f;
}

static void move(const osim* S, real v, real acc, real* dx, real* vn) { move_fl(S, v, acc, dx, vn, NULL); }

/* never advance past the rear of the vehicle ahead */
static int clampmv_fl(lead_t L, real* dx, real* vn, int* fl) {
    if (L.kind != 0 && *dx > L.s) {
        int f = TF_CLAMP;
        if (!(L.s > (real)0)) f |= TF_CLAMP_ZERO;
        if (!(*vn < L.vl)) f |= TF_CLAMP_V;
        *dx = RMAX(L.s, (real)0);
        *vn = RMIN(*vn, L.vl);
        if (fl) *fl |= f;
        return 1;
    }
    return 0;
}

static int clampmv(lead_t L, real* dx, real* vn) { return clampmv_fl(L, dx, vn, NULL); }

/* ------------------------------------------------------------------------ */
/* step                                                                        */
typedef struct {
    int kind;
    real xs, vs;                 /* outcome if the vehicle keeps its place (or loses its claim) */
    int32_t tkey, tedge, tlane;  /* claim target */
    real X, vc, f;               /* front on the target, speed, crossing fraction */
    int32_t lo, hi;              /* claim cells */
    int clamped;
    int lc_eval;  /* passed the lane-change eligibility test */
    real vn;                     /* speed after the own-lane motion */
    int own_fl, chg_fl;          /* branch flags of the own-lane and the lane-change motion */
    int32_t own_lead, chg_lead;  /* vehicle ahead used by each (-1: free road) */
} dec_t;

typedef struct {
    int32_t key, lo, hi, vid, src; /* src: index into the ordered vehicles, or -1-k for insert k */
    int win;
} claim_t;

static int cmp_claim(const void* a, const void* b) {
    const claim_t *u = (const claim_t*)a, *w = (const claim_t*)b;
    if (u->key != w->key) return u->key < w->key ? -1 : 1;
    return (u->vid > w->vid) - (u->vid < w->vid);
}

static void claim_cells(const osim* S, int32_t edge, int32_t ty, real X, int32_t* lo, int32_t* hi) {
    int32_t a = (int32_t)RFLOOR(X - S->tclaim[ty]);
    int32_t b = (int32_t)RFLOOR(X);
    *lo = a < 0 ? 0 : a;
    *hi = b > S->ncell[edge] - 1 ? S->ncell[edge] - 1 : b;
}

typedef struct {
    const osim* S;
    const veh_t* act;
    const int32_t* ord;   /* ordered position -> index in act */
    const int32_t* first; /* lane key -> ordered position of its rearmost vehicle, or -1 */
    const int32_t* cnt;   /* lane key -> number of vehicles */
} view_t;

static const veh_t* at(const view_t* W, int32_t o) { return &W->act[W->ord[o]]; }

/* Is the movement e -> next held at the end of e this step? */
static int blocked(const osim* S, int32_t e, int32_t next, int32_t vid) {
    if (!S->ctrl || next < 0) return 0;
    int32_t h = S->col_idx[e];
    if (S->ctrl[h] == 1) return S->holder[h] != vid;
    if (S->ctrl[h] == 2) {
        int32_t m = S->row_ptr[h + 1] - S->row_ptr[h];
        int32_t phase = (S->t / S->green) % (S->in_deg[h] * m);
        return phase != S->in_rank[e] * m + (next - S->row_ptr[h]);
    }
    return 0;
}

/* a stopped virtual vehicle whose rear is at the link end */
static lead_t stop_line(const osim* S, int32_t e, real x) {
    lead_t L = {3, S->len[e] - x, (real)0, S->len[e], -1, (real)0};
    return L;
}

/* vehicle ahead on lane key k of link e for a vehicle at x (strictly ahead),
 * else the stop line if the vehicle's movement is held, else the rearmost
 * vehicle of lane min(l, lanes-1) of the next link. */
static lead_t lead_in_lane(const view_t* W, int32_t e, int32_t k, real x, int32_t next, int32_t l, int held) {
    const osim* S = W->S;
    lead_t L = {0, 0, 0, 0, -1, 0};
    int32_t f = W->first[k], n = W->cnt[k];
    for (int32_t j = 0; j < n; ++j) {
        const veh_t* q = at(W, f + j);
        if (q->x > x) {
            L.kind = 1; L.xl = q->x; L.vl = q->v; L.ll = S->tlen[q->ty]; L.s = (q->x - L.ll) - x; L.vid = q->vid;
            return L;
        }
    }
    if (held) return stop_line(S, e, x);
    if (next >= 0) {
        int32_t l2 = l < S->lanes[next] - 1 ? l : S->lanes[next] - 1;
        int32_t k2 = lane_key(S, next, l2);
        if (W->cnt[k2] > 0) {
            const veh_t* q = at(W, W->first[k2]);
            L.kind = 2; L.xl = q->x; L.vl = q->v; L.ll = S->tlen[q->ty];
            L.s = (S->len[e] - x) + (q->x - L.ll); L.vid = q->vid;
        }
    }
    return L;
}

/* the same vehicle ahead, seen from another vehicle at xf on the same link */
static lead_t relead(const osim* S, int32_t e, lead_t L, real xf) {
    lead_t R = L;
    if (L.kind == 1) R.s = (L.xl - L.ll) - xf;
    else if (L.kind == 2) R.s = (S->len[e] - xf) + (L.xl - L.ll);
    else if (L.kind == 3) R.s = S->len[e] - xf;
    return R;
}

static dec_t decide(const view_t* W, int32_t o) {
    const osim* S = W->S;
    const veh_t* me = at(W, o);
    int32_t e = me->edge, l = me->lane, c = S->cls[e], k = lane_key(S, e, l), ty = me->ty;
    real len = S->len[e], iv = S->inv_v0[e * S->nt + ty], x = me->x, v = me->v;
    real lme = S->tlen[ty]; /* own length */
    dec_t D;
    memset(&D, 0, sizeof(D));

    /* own leader: the next vehicle of this lane, else look ahead one link */
    const int held = blocked(S, e, me->next, me->vid);
    lead_t L = {0, 0, 0, 0, -1, 0};
    if (o + 1 < S->nact && lane_key(S, at(W, o + 1)->edge, at(W, o + 1)->lane) == k) {
        const veh_t* q = at(W, o + 1);
        L.kind = 1; L.xl = q->x; L.vl = q->v; L.ll = S->tlen[q->ty]; L.s = (q->x - L.ll) - x; L.vid = q->vid;
    } else if (held) {
        L = stop_line(S, e, x);
    } else if (me->next >= 0) {
        int32_t n2 = me->next;
        int32_t l2 = l < S->lanes[n2] - 1 ? l : S->lanes[n2] - 1;
        int32_t k2 = lane_key(S, n2, l2);
        if (W->cnt[k2] > 0) {
            const veh_t* q = at(W, W->first[k2]);
            L.kind = 2; L.xl = q->x; L.vl = q->v; L.ll = S->tlen[q->ty];
            L.s = (len - x) + (q->x - L.ll); L.vid = q->vid;
        }
    }
    D.own_fl = lead_flags(L);
    D.own_lead = L.kind ? L.vid : -1;
    D.chg_lead = -1;
    real ac = idm_fl(S, c, ty, iv, v, L, &D.own_fl);
    real dx, vn;
    move_fl(S, v, ac, &dx, &vn, &D.own_fl);
    D.clamped = clampmv_fl(L, &dx, &vn, &D.own_fl);
    D.vn = vn;
    real xs = x + dx;
    if (xs > len) { /* the front passes the link end strictly */
        real fq = (len - x) / dx;
        if (!(fq < (real)1)) D.own_fl |= TF_F_ONE;
        D.f = dx > (real)0 ? RMIN(fq, (real)1) : (real)0;
        if (me->next < 0) {
            D.kind = K_ARRIVE;
            return D;
        }
        int32_t n2 = me->next;
        D.kind = K_CROSS;
        D.tedge = n2;
        D.tlane = l < S->lanes[n2] - 1 ? l : S->lanes[n2] - 1;
        D.tkey = lane_key(S, n2, D.tlane);
        D.X = xs - len;
        D.vc = vn;
        D.xs = len;
        D.vs = (real)0;
        claim_cells(S, n2, ty, D.X, &D.lo, &D.hi);
        return D;
    }
    D.kind = K_STAY;
    D.xs = xs;
    D.vs = vn;

    /* lane change (Sec. 6.3.2): eligibility */
    int32_t n = S->lanes[e];
    if (n < 2 || (S->t - me->lc) < S->lc_cool || x < lme) return D;
    D.lc_eval = 1;
    int32_t lo = 0, hi = n - 1;
    if (me->next >= 0) {
        int32_t hn = S->col_idx[e];
        int32_t m = S->row_ptr[hn + 1] - S->row_ptr[hn];
        int32_t j = me->next - S->row_ptr[hn];
        lo = (j * n) / m;
        hi = ((j + 1) * n + m - 1) / m - 1;
        if (hi < lo) hi = lo;
    }
    real d = len - x;
    int inband = lo <= l && l <= hi;
    int mand = !inband && d <= S->dmand;
    int32_t cand[2];
    int nc = 0;
    if (mand) {
        cand[nc++] = l < lo ? l + 1 : l - 1;
    } else {
        for (int32_t s = l - 1; s <= l + 1; s += 2) {
            if (s < 0 || s >= n) continue;
            if (inband && d <= S->dmand && (s < lo || s > hi)) continue;
            cand[nc++] = s;
        }
    }
    /* follower in the own lane (same link) */
    const veh_t* F = NULL;
    if (o > 0 && lane_key(S, at(W, o - 1)->edge, at(W, o - 1)->lane) == k) F = at(W, o - 1);

    int best = -1, best_fl = 0;
    int32_t best_lead = -1;
    real best_inc = 0, best_X = 0, best_v = 0;
    for (int ci = 0; ci < nc; ++ci) {
        int32_t lt = cand[ci], kt = lane_key(S, e, lt);
        lead_t Lt = lead_in_lane(W, e, kt, x, me->next, lt, held);
        /* lag: last vehicle of the target lane with position <= x */
        const veh_t* Ft = NULL;
        for (int32_t j = 0; j < W->cnt[kt]; ++j) {
            const veh_t* q = at(W, W->first[kt] + j);
            if (q->x <= x) Ft = q; else break;
        }
        /* gap acceptance */
        if (Lt.kind != 0 && Lt.s < S->s0) continue;
        if (Ft && ((x - lme) - Ft->x) < S->s0) continue;
        int tfl = lead_flags(Lt);
        real at_ = idm_fl(S, c, ty, iv, v, Lt, &tfl);
        if (at_ < -S->bsafe) continue;
        real dxt, vt;
        move_fl(S, v, at_, &dxt, &vt, &tfl);
        clampmv_fl(Lt, &dxt, &vt, &tfl);
        real Xt = x + dxt;
        if (Xt >= len) continue;
        real an = 0, ant = 0;
        if (Ft) {
            const int32_t tf = Ft->ty; /* the lag follows with its own type's constants */
            const real ivf = S->inv_v0[e * S->nt + tf];
            an = idm(S, c, tf, ivf, Ft->v, relead(S, e, Lt, Ft->x));
            lead_t Li = {1, (x - lme) - Ft->x, v, x, me->vid, lme};
            ant = idm(S, c, tf, ivf, Ft->v, Li);
            if (ant < -S->bsafe) continue;
            lead_t none = {0, 0, 0, 0, -1, 0};
            real afree = idm(S, c, tf, ivf, Ft->v, none);
            real dxF, vF;
            move(S, Ft->v, afree, &dxF, &vF);
            if (((Xt - lme) - Ft->x) < dxF) continue;
        }
        real inc = 0;
        if (!mand) {
            real d1 = at_ - ac;
            real d2 = Ft ? (ant - an) : (real)0;
            real d3 = (real)0;
            if (F) {
                const int32_t tf = F->ty;
                const real ivf = S->inv_v0[e * S->nt + tf];
                lead_t Lo = {1, (x - lme) - F->x, v, x, me->vid, lme};
                real ao = idm(S, c, tf, ivf, F->v, Lo);
                real aot = idm(S, c, tf, ivf, F->v, relead(S, e, L, F->x));
                d3 = aot - ao;
            }
            inc = d1 + S->p * (d2 + d3);
            if (!(inc > S->athr)) continue;
        }
        if (best < 0 || inc > best_inc) {
            best = lt; best_inc = inc; best_X = Xt; best_v = vt;
            best_fl = tfl; best_lead = Lt.kind ? Lt.vid : -1;
        }
    }
    if (best >= 0) {
        D.kind = K_CHANGE;
        D.tedge = e;
        D.tlane = best;
        D.tkey = lane_key(S, e, best);
        D.X = best_X;
        D.vc = best_v;
        D.chg_fl = best_fl;
        D.chg_lead = best_lead;
        claim_cells(S, e, ty, best_X, &D.lo, &D.hi);
    }
    return D;
}

/* Fuel and CO over one step (Sec. 6.3.4): the fuel-consumption equation with
 * v in m/s and the realized acceleration a = (v' - v)/dt, its bracket floored
 * at 0 (fuel never below idle), P_ea = 0.79296 a^2 v only while accelerating;
 * the CO equation with v in miles per hour; both rates integrated over dt. */
static void emissions(const osim* S, veh_t* q, real v1) {
    real v = q->v;
    real a = (v1 - v) / S->dt;
    real vm = v * S->mph;
    real d = vm - (real)50;
    real c = (real)-0.064 + (real)0.0056 * vm + (real)0.00026 * (d * d);
    real pea = a > (real)0 ? ((real)0.79296 * (a * a)) * v : (real)0;
    real br = (real)0.269 * v + (real)0.0171 * (v * v) + (real)0.000672 * ((v * v) * v) + (real)1.680 * (a * v) + pea;
    br = RMAX(br, (real)0);
    real f = (real)0.666 + (real)0.072 * br;
    q->fuel = q->fuel + f * S->dt;
    q->co = q->co + c * S->dt;
}

static void record_exit(osim* S, const veh_t* q, real f, int32_t t) {
    int64_t ns = (int64_t)(t + 1) - q->kin;
    real frac = f - q->phin;
    S->st_cnt[q->edge] += 1;
    S->st_steps[q->edge] += ns;
    S->st_us[q->edge] += ns * S->dt_us + (int64_t)RRINT(frac * S->dt_us_f);
}

static int step_once(osim* S) {
    int32_t t = S->t, N = S->nact;
    int32_t *ord = (int32_t*)malloc(sizeof(int32_t) * (N + 1));
    int32_t *first = (int32_t*)malloc(sizeof(int32_t) * (S->nlanes + 1));
    int32_t *cnt = (int32_t*)calloc(S->nlanes + 1, sizeof(int32_t));
    for (int32_t i = 0; i < N; ++i) ord[i] = i;
    g_S = S; g_act = S->act;
    qsort(ord, N, sizeof(int32_t), cmp_order);
    for (int32_t k = 0; k < S->nlanes; ++k) first[k] = -1;
    for (int32_t o = 0; o < N; ++o) {
        const veh_t* q = &S->act[ord[o]];
        int32_t k = lane_key(S, q->edge, q->lane);
        if (first[k] < 0) first[k] = o;
        cnt[k] += 1;
    }
    view_t W = {S, S->act, ord, first, cnt};

    /* stop control: a free stop node admits the lowest-id vehicle waiting at
     * its line (front within stop_dist of the link end, speed <= stop_speed,
     * going on to another link) */
    if (S->ctrl) {
        /* a pending choice is kept as -2 - vid until every vehicle is seen */
        for (int32_t o = 0; o < N; ++o) {
            const veh_t* q = at(&W, o);
            int32_t h = S->col_idx[q->edge];
            if (S->ctrl[h] != 1 || q->next < 0 || S->holder[h] >= 0) continue;
            if (!((S->len[q->edge] - q->x) <= S->stop_dist) || !(q->v <= S->stop_speed)) continue;
            if (S->holder[h] == -1 || q->vid < -2 - S->holder[h]) S->holder[h] = -2 - q->vid;
        }
        for (int32_t u = 0; u < S->nn; ++u)
            if (S->holder[u] <= -2) S->holder[u] = -2 - S->holder[u];
    }

    /* utilization / speed sample of the state at t (Sec. 6.4) */
    if (S->samp_every > 0 && t % S->samp_every == 0) {
        int32_t g = (t / S->samp_every) / S->samp_group;
        if (g < S->samp_max) {
            for (int32_t o = 0; o < N; ++o) {
                const veh_t* q = at(&W, o);
                S->samp_cnt[(int64_t)g * S->ne + q->edge] += 1;
                S->samp_spd[(int64_t)g * S->ne + q->edge] += (int64_t)RRINT(q->v * (real)1e6);
            }
        }
    }

    /* 1. decisions of the vehicles on the road */
    dec_t* D = (dec_t*)malloc(sizeof(dec_t) * (N + 1));
    /* each decision reads state t only: the all-cores build (-fopenmp) splits
     * this loop over threads, with the same result */
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t o = 0; o < N; ++o) D[o] = decide(&W, o);

    /* 2. insertion candidates: waiting trips due now, in vehicle-id order */
    int32_t ncand = S->npend;
    int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (S->npend + S->ntrips + 1));
    memcpy(cand, S->pend, sizeof(int32_t) * S->npend);
    while (S->relc < S->ntrips && S->dep[S->relc] < t) S->relc += 1;
    for (int32_t v = S->relc; v < S->ntrips && S->dep[v] == t; ++v)
        if (S->depart_actual[v] < 0) cand[ncand++] = v;
    int32_t* clane = (int32_t*)malloc(sizeof(int32_t) * (ncand + 1));

    /* 3. claims */
    claim_t* C = (claim_t*)malloc(sizeof(claim_t) * (N + ncand + 1));
    int32_t nclaim = 0;
    for (int32_t o = 0; o < N; ++o) {
        if (D[o].kind == K_CROSS || D[o].kind == K_CHANGE) {
            claim_t c = {D[o].tkey, D[o].lo, D[o].hi, at(&W, o)->vid, o, 0};
            C[nclaim++] = c;
            if (D[o].kind == K_CHANGE) S->claims_lc += 1;
        }
        S->lc_evaluated += D[o].lc_eval;
    }
    const int32_t nclaim_veh = nclaim;
    for (int32_t i = 0; i < ncand; ++i) {
        int32_t v = cand[i];
        int32_t e0 = S->route_edges[S->rbeg[v]];
        int32_t best = -1;
        real bsp = 0;
        for (int32_t l = 0; l < S->lanes[e0]; ++l) {
            int32_t k = lane_key(S, e0, l);
            real sp = cnt[k] > 0 ? (at(&W, first[k])->x - S->tlen[at(&W, first[k])->ty]) : S->len[e0];
            if (best < 0 || sp > bsp) { best = l; bsp = sp; }
        }
        clane[i] = -1;
        if (bsp >= S->tclaim[S->vtype[v]]) {
            clane[i] = best;
            claim_t c;
            c.key = lane_key(S, e0, best);
            claim_cells(S, e0, S->vtype[v], S->tlen[S->vtype[v]], &c.lo, &c.hi);
            c.vid = v; c.src = -1 - i; c.win = 0;
            C[nclaim++] = c;
        }
    }
    S->claims += nclaim;
    S->claims_dep += nclaim - nclaim_veh;
    /* a claim wins iff no overlapping claim on the same lane has a lower id */
    qsort(C, nclaim, sizeof(claim_t), cmp_claim);
    int32_t* cwin_veh = (int32_t*)calloc(N + 1, sizeof(int32_t));
    int32_t* cwin_ins = (int32_t*)calloc(ncand + 1, sizeof(int32_t));
    for (int32_t a = 0; a < nclaim;) {
        int32_t b = a;
        while (b < nclaim && C[b].key == C[a].key) ++b;
        for (int32_t i = a; i < b; ++i) {
            int win = 1;
            for (int32_t j = a; j < b; ++j) {
                if (C[j].vid < C[i].vid && C[j].lo <= C[i].hi && C[i].lo <= C[j].hi) { win = 0; break; }
            }
            C[i].win = win;
            if (!win) S->claims_lost += 1;
            if (C[i].src >= 0) cwin_veh[C[i].src] = win;
            else cwin_ins[-1 - C[i].src] = win;
        }
        a = b;
    }

    /* 4. apply */
    veh_t* nact = (veh_t*)malloc(sizeof(veh_t) * (N + ncand + 1));
    int32_t nn = 0;
    for (int32_t o = 0; o < N; ++o) {
        veh_t q = *at(&W, o);
        const dec_t* d = &D[o];
        S->clamps += d->clamped;
        if (S->tape_on) {
            int32_t mode = TM_STAY, lead = d->own_lead, fl = d->own_fl;
            if (d->kind == K_ARRIVE) mode = TM_ARRIVE;
            else if (d->kind == K_CROSS) mode = cwin_veh[o] ? TM_CROSS : TM_YIELD;
            else if (d->kind == K_CHANGE && cwin_veh[o]) { mode = TM_CHANGE; lead = d->chg_lead; fl = d->chg_fl; }
            tape_push(S, t, q.vid, mode, lead, fl, q.edge, (double)q.x, (double)q.v);
        }
        if (d->kind == K_ARRIVE) {
            record_exit(S, &q, d->f, t);
            emissions(S, &q, d->vn);
            S->fuel_total[q.vid] = q.fuel;
            S->co_total[q.vid] = q.co;
            S->arrive_step[q.vid] = t + 1;
            S->arrived += 1;
            continue;
        }
        {
            real v1 = d->vs; /* the speed the vehicle ends the step with */
            if (d->kind == K_CROSS && cwin_veh[o]) v1 = d->vc;
            else if (d->kind == K_CHANGE && cwin_veh[o]) v1 = d->vc;
            emissions(S, &q, v1);
        }
        if (d->kind == K_CROSS && cwin_veh[o]) {
            if (S->ctrl && S->holder[S->col_idx[q.edge]] == q.vid) S->holder[S->col_idx[q.edge]] = -1;
            record_exit(S, &q, d->f, t);
            q.rcur += 1;
            q.edge = d->tedge;
            q.lane = d->tlane;
            q.next = (q.rcur + 1 < S->rend[q.vid]) ? S->route_edges[q.rcur + 1] : -1;
            q.x = d->X;
            q.v = d->vc;
            q.kin = t + 1;
            q.phin = d->f;
        } else if (d->kind == K_CHANGE && cwin_veh[o]) {
            q.lane = d->tlane;
            q.x = d->X;
            q.v = d->vc;
            q.lc = t;
        } else {
            q.x = d->xs;
            q.v = d->vs;
        }
        nact[nn++] = q;
    }
    int32_t np = 0;
    for (int32_t i = 0; i < ncand; ++i) {
        int32_t v = cand[i];
        if (clane[i] >= 0 && cwin_ins[i]) {
            veh_t q;
            q.vid = v;
            q.rcur = S->rbeg[v];
            q.edge = S->route_edges[q.rcur];
            q.lane = clane[i];
            q.next = (q.rcur + 1 < S->rend[v]) ? S->route_edges[q.rcur + 1] : -1;
            q.ty = S->vtype[v];
            q.x = S->tlen[q.ty];
            q.v = (real)0;
            q.lc = LC_NONE;
            q.kin = t + 1;
            q.phin = (real)1;
            q.fuel = (real)0;
            q.co = (real)0;
            nact[nn++] = q;
            S->depart_actual[v] = t + 1;
            S->departed += 1;
            tape_push(S, t + 1, v, TM_APPEAR, -1, 0, q.edge, (double)q.x, (double)q.v);
        } else {
            S->pend[np++] = v;
        }
    }
    S->npend = np;
    S->updates += N;
    free(S->act);
    S->act = nact;
    S->nact = nn;
    S->t = t + 1;
    free(ord); free(first); free(cnt); free(D); free(cand); free(clane); free(C);
    free(cwin_veh); free(cwin_ins);
    return OR_OK;
}

int or_step(osim* S, int32_t n) {
    if (!S->loaded) return OR_ESTATE;
    for (int32_t i = 0; i < n; ++i) {
        int rc = step_once(S);
        if (rc) return rc;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* outputs                                                                     */
/* counters: step, loaded, waiting, en_route, arrived, departed, vehicle_updates,
 * claims_lost, clamps, claims, claims_departure, lc_evaluated, claims_lane_change */
void or_counters(const osim* S, int64_t* out) {
    out[0] = S->t;
    out[1] = S->ntrips;
    out[2] = (int64_t)S->ntrips - S->departed;
    out[3] = S->nact;
    out[4] = S->arrived;
    out[5] = S->departed;
    out[6] = S->updates;
    out[7] = S->claims_lost;
    out[8] = S->clamps;
    out[9] = S->claims;
    out[10] = S->claims_dep;
    out[11] = S->lc_evaluated;
    out[12] = S->claims_lc;
}

static int cmp_vid(const void* a, const void* b) {
    const veh_t *u = (const veh_t*)a, *w = (const veh_t*)b;
    return (u->vid > w->vid) - (u->vid < w->vid);
}

/* active vehicles sorted by vehicle id; ints: vid, edge, lane, cursor (index
 * in the route), lc, kin; reals (as double): x, v, phin, fuel, co */
int32_t or_get_vehicles(osim* S, int32_t* iv, double* rv) {
    qsort(S->act, S->nact, sizeof(veh_t), cmp_vid);
    for (int32_t i = 0; i < S->nact; ++i) {
        const veh_t* q = &S->act[i];
        iv[6 * i + 0] = q->vid;
        iv[6 * i + 1] = q->edge;
        iv[6 * i + 2] = q->lane;
        iv[6 * i + 3] = q->rcur - S->rbeg[q->vid];
        iv[6 * i + 4] = q->lc;
        iv[6 * i + 5] = q->kin;
        rv[5 * i + 0] = (double)q->x;
        rv[5 * i + 1] = (double)q->v;
        rv[5 * i + 2] = (double)q->phin;
        rv[5 * i + 3] = (double)q->fuel;
        rv[5 * i + 4] = (double)q->co;
    }
    return S->nact;
}

void or_get_emissions(const osim* S, double* fuel, double* co) {
    for (int32_t v = 0; v < S->ntrips; ++v) {
        fuel[v] = (double)S->fuel_total[v];
        co[v] = (double)S->co_total[v];
    }
}

int or_set_sampler(osim* S, int32_t every, int32_t group, int32_t max_groups) {
    if (every <= 0 || group <= 0 || max_groups <= 0) return OR_EINVAL;
    free(S->samp_cnt);
    free(S->samp_spd);
    S->samp_every = every;
    S->samp_group = group;
    S->samp_max = max_groups;
    S->samp_cnt = (int64_t*)calloc((size_t)max_groups * S->ne, sizeof(int64_t));
    S->samp_spd = (int64_t*)calloc((size_t)max_groups * S->ne, sizeof(int64_t));
    return OR_OK;
}

void or_get_samples(const osim* S, int64_t* cnt, int64_t* spd) {
    memcpy(cnt, S->samp_cnt, sizeof(int64_t) * (size_t)S->samp_max * S->ne);
    memcpy(spd, S->samp_spd, sizeof(int64_t) * (size_t)S->samp_max * S->ne);
}

void or_get_trips(const osim* S, int32_t* depart_actual, int32_t* arrive_step) {
    memcpy(depart_actual, S->depart_actual, sizeof(int32_t) * S->ntrips);
    memcpy(arrive_step, S->arrive_step, sizeof(int32_t) * S->ntrips);
}

void or_get_edge_stats(const osim* S, int64_t* cnt, int64_t* steps, int64_t* us) {
    memcpy(cnt, S->st_cnt, sizeof(int64_t) * S->ne);
    memcpy(steps, S->st_steps, sizeof(int64_t) * S->ne);
    memcpy(us, S->st_us, sizeof(int64_t) * S->ne);
}

int32_t or_num_active(const osim* S) { return S->nact; }

/* event tape: recording switch, size, copy-out (records in step order; at one
 * step, the vehicles that appear come before the moves of that step only in
 * the sense that APPEAR records carry the state index at which they appear) */
void or_tape_enable(osim* S, int32_t on) { S->tape_on = on; }
int64_t or_tape_size(const osim* S) { return S->tp_n; }
void or_tape_get(const osim* S, int32_t* step, int32_t* vid, int32_t* mode, int32_t* lead, int32_t* flags,
                 int32_t* edge, double* x0, double* v0) {
    int64_t n = S->tp_n;
    memcpy(step, S->tp_step, sizeof(int32_t) * n);
    memcpy(vid, S->tp_vid, sizeof(int32_t) * n);
    memcpy(mode, S->tp_mode, sizeof(int32_t) * n);
    memcpy(lead, S->tp_lead, sizeof(int32_t) * n);
    memcpy(flags, S->tp_flags, sizeof(int32_t) * n);
    memcpy(edge, S->tp_edge, sizeof(int32_t) * n);
    memcpy(x0, S->tp_x0, sizeof(double) * n);
    memcpy(v0, S->tp_v0, sizeof(double) * n);
}
int32_t or_num_pending(const osim* S) { return S->npend; }

/* Continue from a state taken from another simulation of the same network,
 * parameters, vehicle types and demand at step t (after or_load_demand, before
 * any step, no intersection control):
 *   n vehicles on the road, ints iv[6n] = (vid, edge, lane, cursor in the
 *   route, step of the last lane change, entry step), reals rv[5n] as float =
 *   (x, v, entry fraction, fuel, co);
 *   per vehicle id: depart_actual, arrive_step, fuel_total, co_total;
 *   per link: traversal count, whole steps, interpolated microseconds;
 *   counters[13] in the order of or_counters.
 * The trips still waiting are those not on the road whose departure step is
 * before t; they queue in vehicle-id order, as they would have. */
int or_set_state(osim* S, int32_t t, int32_t n, const int32_t* iv, const double* rv, const int32_t* depart_actual,
                 const int32_t* arrive_step, const double* fuel_total, const double* co_total, const int64_t* cnt,
                 const int64_t* steps, const int64_t* us, const int64_t* counters) {
    if (!S->loaded || S->ctrl || S->t != 0 || t < 0 || n < 0 || n > S->ntrips) return OR_ESTATE;
    for (int32_t i = 0; i < n; ++i) {
        int32_t vid = iv[6 * i + 0], e = iv[6 * i + 1], l = iv[6 * i + 2], cur = iv[6 * i + 3];
        if (vid < 0 || vid >= S->ntrips || cur < 0 || S->rbeg[vid] + cur >= S->rend[vid]) return OR_EINVAL;
        if (S->route_edges[S->rbeg[vid] + cur] != e || l < 0 || l >= S->lanes[e]) return OR_EINVAL;
        if (!(rv[5 * i + 0] >= 0) || !(rv[5 * i + 0] <= (double)S->len[e]) || !(rv[5 * i + 1] >= 0)) return OR_EINVAL;
    }
    for (int32_t i = 0; i < n; ++i) {
        veh_t* q = &S->act[i];
        q->vid = iv[6 * i + 0];
        q->edge = iv[6 * i + 1];
        q->lane = iv[6 * i + 2];
        q->rcur = S->rbeg[q->vid] + iv[6 * i + 3];
        q->next = (q->rcur + 1 < S->rend[q->vid]) ? S->route_edges[q->rcur + 1] : -1;
        q->lc = iv[6 * i + 4];
        q->kin = iv[6 * i + 5];
        q->ty = S->vtype[q->vid];
        q->x = (real)rv[5 * i + 0];
        q->v = (real)rv[5 * i + 1];
        q->phin = (real)rv[5 * i + 2];
        q->fuel = (real)rv[5 * i + 3];
        q->co = (real)rv[5 * i + 4];
    }
    S->nact = n;
    for (int32_t v = 0; v < S->ntrips; ++v) {
        S->depart_actual[v] = depart_actual[v];
        S->arrive_step[v] = arrive_step[v];
        S->fuel_total[v] = (real)fuel_total[v];
        S->co_total[v] = (real)co_total[v];
    }
    memcpy(S->st_cnt, cnt, sizeof(int64_t) * S->ne);
    memcpy(S->st_steps, steps, sizeof(int64_t) * S->ne);
    memcpy(S->st_us, us, sizeof(int64_t) * S->ne);
    S->npend = 0;
    for (int32_t v = 0; v < S->ntrips; ++v)
        if (S->dep[v] < t && S->depart_actual[v] < 0) S->pend[S->npend++] = v;
    S->relc = 0;
    S->t = t;
    S->arrived = counters[4];
    S->departed = counters[5];
    S->updates = counters[6];
    S->claims_lost = counters[7];
    S->clamps = counters[8];
    S->claims = counters[9];
    S->claims_dep = counters[10];
    S->lc_evaluated = counters[11];
    S->claims_lc = counters[12];
    return OR_OK;
}
