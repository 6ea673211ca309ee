// The kernels of one synchronous simulation step (included once, by
// trafficsim.hip).  See trafficsim.hip for the overview.
#pragma once

#include "common.h"

namespace tsim {
// first j in [lo, hi) with x[j] > X (x sorted ascending within a lane)
__device__ __forceinline__ int ub_x(const float* __restrict__ x, int lo, int hi, float X) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (x[mid] <= X) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first j in [lo, hi) with x[j] >= X
__device__ __forceinline__ int lb_x(const float* __restrict__ x, int lo, int hi, float X) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (x[mid] < X) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// k_decide
// ---------------------------------------------------------------------------
// A block takes the sorted entries in tiles (of its threads times the entries
// per thread).  The tile and H entries on either side sit in LDS, slot s
// holding entry b0 - H + s: the vehicle
// ahead of an entry in its lane, the one behind it, and the run of a
// neighbouring lane (the lanes of a link are consecutive keys, so their runs
// are next to the entry's own) are then LDS reads.  The H entries beyond each
// end keep the runs that cross the tile's ends in LDS too: without them the
// waves at both ends of every tile would search such runs in global memory,
// and the block, which waits for its slowest wave, with them.  A slot before
// the first entry holds key -1 and a slot past the last entry key INT_MAX, so
// the keys stay sorted over the whole window.
constexpr int kTileHalo = 32;
template <int NS, int H>
struct Tile {
    static constexpr int kSlots = NS;
    static constexpr int kHalo = H;
    int key[NS];
    float x[NS];
    float v[NS];
    int ty[NS];
};
constexpr int kKeyPast = 0x7FFFFFFF;

// What the lane-change evaluation of a vehicle takes over from its step
// decision: its entry, link records, own leader and own-lane acceleration.
struct Own {
    int i, k, e, nx, ty, vid, l;
    float x, v, lme, ac;
    bool held, front;
    DrvRec D;
    EdgeRec E2;  // next link's record: read by front vehicles only
    Lead L;
};

// The claims of a block's vehicles (crossings and lane changes, at most one per
// vehicle), gathered in LDS while its tiles are decided and issued together
// when the stage is more than half full and after the block's last tile: the
// chain of a claim (its link's claim record, the cell atomics, the list slot)
// is waited for once every few tiles instead of once for every pass of a wave
// that holds a claiming vehicle.  NT is twice the tile, so a tile's claims
// always fit.
template <int NT>
struct ClaimStage {
    int n;
    int i[NT];      // entry of the claiming vehicle
    int tedge[NT];  // target link
    int pk[NT];     // target lane | kind << 8 | type << 16
    float X[NT], v[NT], f[NT];
};

template <class StageT>
__device__ __forceinline__ void stage_claim(StageT& CS, int i, int tedge, int tlane, int kind, int ty, float X, float v,
                                            float f) {
    const int m = atomicAdd(&CS.n, 1);
    CS.i[m] = i;
    CS.tedge[m] = tedge;
    CS.pk[m] = tlane | (kind << 8) | (ty << 16);
    CS.X[m] = X;
    CS.v[m] = v;
    CS.f[m] = f;
}

// issues the staged claims (after a barrier that follows the last
// stage_claim): their cells, then their slots in segment seg of the list; the
// claimant's id and the target link's first lane are read here
template <int BS, class StageT>
__device__ __forceinline__ void issue_claims(const Params& P, const Net& net, const Veh& in, const Scratch& s,
                                             StageT& CS, int seg, unsigned long long tag) {
    const int M = CS.n;
    for (int m = threadIdx.x; m < M; m += BS) {
        const int te = CS.tedge[m];
        const int pk = CS.pk[m];
        const float X = CS.X[m];
        const int i = CS.i[m];
        const ClaimRec C = net.cr[te];
        const int lb = net.lane_base[te], vid = in.vid[i];
        int lo, hi;
        claim_cells(P, C.ncell, pk >> 16, X, lo, hi);
        push_claim(s, C, lb, seg, tag, vid, (pk >> 8) & 0xFF, i, te, pk & 0xFF, X, CS.v[m], CS.f[m], lo, hi);
    }
}

// Own leader: the next entry if it is in the same lane (ka, xa, va, tya), else
// the stop line if the movement at the link end is held, else the rearmost
// vehicle of the mapped lane of the next link of the route (E2), if any.
__device__ __forceinline__ Lead own_leader(const Params& P, const Scratch& s, unsigned ep, int i, int N, int k,
                                           float x, float len, int l, bool held, int nx, const EdgeRec& E2, int ka,
                                           float xa, float va, int tya) {
    Lead L = {0, 0.0f, 0.0f, 0.0f, -1, 0.0f};
    if (i + 1 < N && ka == k) {
        L.kind = 1; L.xl = xa; L.vl = va; L.ll = by_type(P.tlen, tya); L.s = (xa - L.ll) - x; L.idx = i + 1;
    } else if (held) {
        L = stop_line_lead(len, x);
    } else if (nx >= 0) {
        int nl2 = E2.lanes;
        int k2 = E2.lane_base + (l < nl2 - 1 ? l : nl2 - 1);
        int j, tyr;
        float xl, vr;
        // selects, not a branch: the lane record is then read whole at once
        const bool ok = lane_rear(s.lanes, k2, ep, j, xl, vr, tyr);
        const float ll = by_type(P.tlen, tyr);
        L.kind = ok ? 2 : 0;
        L.xl = ok ? xl : 0.0f;
        L.vl = ok ? vr : 0.0f;
        L.ll = ok ? ll : 0.0f;
        L.s = ok ? (len - x) + (xl - ll) : 0.0f;
        L.idx = ok ? j : -1;
    }
    return L;
}

// The step decision of entry i (tile slot t_slot): leader, IDM, move, crossing
// claim or arrival.  Returns true when the vehicle is to be evaluated for a
// lane change, with what that needs in o.
template <bool kFull, class TileT, class StageT>
__device__ bool decide_vehicle(const Params& P, const Net& net, const Trips& tr, const Veh& in, const Scratch& s,
                               const Tape& tp, const TileT& T, StageT& CS, int t_slot, int N, int t, unsigned ep,
                               unsigned long long tag, int i, int e, int nx, int vid, int lcs, int& clamps,
                               int& arrivals, Own& o) {
    // the own entry and the one after it from the tile; the records of the
    // own link and type, and for the front vehicle of a lane the next link's,
    // issued before the first branch
    const int k = T.key[t_slot];
    const float x = T.x[t_slot];
    const float v = T.v[t_slot];
    const int ty = T.ty[t_slot];
    const int ka = T.key[t_slot + 1];
    const float xa = T.x[t_slot + 1], va = T.v[t_slot + 1];
    const int tya = T.ty[t_slot + 1];
    const int nt = P.nt;
    const bool front = !(i + 1 < N && ka == k);
    const DrvRec D = net.drv[e * nt + ty];
    EdgeRec E2 = {0.0f, 0, 1, 0};
    if (front) E2 = net.er[nx >= 0 ? nx : e];
    const float len = D.len;
    const float lme = by_type(P.tlen, ty);  // own length
    const float iv = D.iv, A = D.A, Tg = D.T, kab = D.kab;
    const int lb = D.lane_base;
    const int nlanes = D.lanes_m & 0xFFFF;
    const int l = k - lb;

    const bool held = kFull && movement_held(P, net, s, e, nx, vid, t, tag);
    Lead L = own_leader(P, s, ep, i, N, k, x, len, l, held, nx, E2, ka, xa, va, tya);
    int own_fl = lead_flags(L);
    const float ac = idm_acc_fl(P, A, Tg, kab, iv, v, L, own_fl);
    float dx, vn;
    kin_move_fl(P, v, ac, dx, vn, own_fl);
    clamps += clamp_to_leader_fl(L, dx, vn, own_fl);
    const float xs = x + dx;
    // utilization / speed sample of the state at t (Sec. 6.4)
    if (kFull && s.samp_every > 0 && t % s.samp_every == 0) {
        const int g = (t / s.samp_every) / s.samp_group;
        if (g < s.samp_max) {
            const size_t so = (size_t)g * (size_t)net.ne + (size_t)e;
            atomicAdd(s.samp_cnt + so, 1ull);
            atomicAdd(s.samp_spd + so, (unsigned long long)(long long)rintf(v * 1e6f));
        }
    }
    if (kFull && tp.on) {
        tp.x[i] = x;
        tp.v[i] = v;
        tp.vid[i] = vid;
        tp.edge[i] = e;
        tp.lead[i] = L.idx;
        tp.clead[i] = -1;
        tp.cflags[i] = 0;
        tp.next[i] = -1;
        tp.mode[i] = kModeStay;
    }

    if (xs > len) {  // the front passes the link end strictly (only a lane's front vehicle can)
        float fq = (len - x) / dx;
        if (!(fq < 1.0f)) own_fl |= kFFOne;
        float f = dx > 0.0f ? fmn(fq, 1.0f) : 0.0f;
        if (kFull && tp.on) {
            tp.flags[i] = (unsigned short)own_fl;
            tp.mode[i] = nx < 0 ? kModeArrive : kModeCross;
        }
        if (nx < 0) {  // arrival at the end of the last link
            record_exit(P, s, e, tr.kin[vid], tr.phin[vid], f, t);
            float fu = in.fuel[i], co = in.co[i];
            emissions(P, v, vn, fu, co);
            tr.fuel_total[vid] = fu;
            tr.co_total[vid] = co;
            tr.arrive_step[vid] = t + 1;
            s.stay[i] = 0;
            arrivals += 1;
            return false;
        }
        int nl2 = E2.lanes;
        int tl = l < nl2 - 1 ? l : nl2 - 1;
        float X = xs - len;
        s.xs[i] = len;  // outcome if the claim is lost: wait at the link end
        s.vs[i] = 0.0f;
        s.stay[i] = 1;
        stage_claim(CS, i, nx, tl, kCross, ty, X, vn, f);
        return false;
    }
    s.xs[i] = xs;
    s.vs[i] = vn;
    s.stay[i] = 1;
    if (kFull && tp.on) tp.flags[i] = (unsigned short)own_fl;

    // lane change (Sec. 6.3.2): a vehicle past the cool-down on a multi-lane
    // link that is not on its entry cells
    if (nlanes < 2 || (t - lcs) < P.lc_cool || x < lme) return false;
    o.i = i; o.k = k; o.e = e; o.nx = nx; o.ty = ty; o.vid = vid; o.l = l;
    o.x = x; o.v = v; o.lme = lme; o.ac = ac;
    o.held = held; o.front = front;
    o.D = D; o.E2 = E2; o.L = L;
    return true;
}

// Lane-change evaluation of a vehicle (Sec. 6.3.2): candidate lanes (the
// mandatory one when the vehicle is outside its turn band near the link
// end, else the neighbours inside the band), gap acceptance, the safety
// criterion for the new follower, the incentive criterion; the best candidate
// claims its cells in the target lane.  The follower comes from LDS; a
// target lane's run from the lane index (one record read), and its leader and
// lag from LDS when the tile holds the run, else from the sorted arrays.
template <bool kFull, class TileT, class StageT>
__device__ bool change_vehicle(const Params& P, const Net& net, const Veh& in, const Scratch& s, const Tape& tp,
                               const TileT& T, StageT& CS, int t_slot, int b0, unsigned ep, const Own& o) {
    const int i = o.i, k = o.k, e = o.e, nx = o.nx, ty = o.ty, vid = o.vid, l = o.l;
    const float x = o.x, v = o.v, lme = o.lme, ac = o.ac;
    const bool held = o.held;
    const DrvRec& D = o.D;
    const Lead& L = o.L;
    const int nt = P.nt;
    const int kb = T.key[t_slot - 1];
    const float xb = T.x[t_slot - 1], vb = T.v[t_slot - 1];
    const int tyb = T.ty[t_slot - 1];
    const bool hasF = i > 0 && kb == k;
    // the follower's driver constants: the own record when the types agree
    DrvRec Db = D;
    if (hasF && tyb != ty) Db = net.drv[e * nt + tyb];
    const int m = D.lanes_m >> 16;
    const float len = D.len;
    const float iv = D.iv, A = D.A, Tg = D.T, kab = D.kab;
    const int lb = D.lane_base;
    const int n = D.lanes_m & 0xFFFF;
    int blo = 0, bhi = n - 1;
    if (nx >= 0) {
        const int r0 = D.r0;
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
    const float xF = hasF ? xb : 0.0f;
    const float vF = hasF ? vb : 0.0f;
    EdgeRec E2 = o.E2;
    bool haveE2 = o.front;

    int best = -1, best_fl = 0, best_lead = -1;
    float best_inc = 0.0f, best_X = 0.0f, best_v = 0.0f;
    for (int ci = 0; ci < nc; ++ci) {
        const int lt = cand[ci];
        const int kt = lb + lt;
        // first vehicle of the target lane strictly ahead (position > x) and
        // the one before it, the lag
        bool hasLead = false, hasFt = false;
        int jl = -1;
        float xl = 0.0f, vl = 0.0f, xFt = 0.0f, vFt = 0.0f;
        int tyl = 0, tyFt = 0;
        // the run from the lane index; searched in LDS when the tile holds it
        int tlo, thi;
        const bool occ = lane_range(s.lanes, kt, ep, tlo, thi);
        const int w0 = b0 - TileT::kHalo;  // the entry in slot 0
        if (occ && tlo >= w0 && thi <= w0 + TileT::kSlots - 1) {
            const int ra = tlo - w0, rb = thi - w0;
            int a = ra, c = rb + 1;  // first slot in the run with x > own x
            while (a < c) {
                const int mid = (a + c) >> 1;
                if (T.x[mid] <= x) a = mid + 1;
                else c = mid;
            }
            hasLead = a <= rb;
            hasFt = a - 1 >= ra;
            const int sl = hasLead ? a : t_slot, sf = hasFt ? a - 1 : t_slot;
            jl = w0 + a;
            xl = T.x[sl]; vl = T.v[sl]; tyl = T.ty[sl];
            xFt = T.x[sf]; vFt = T.v[sf]; tyFt = T.ty[sf];
        } else {
            const int j = occ ? ub_x(in.x, tlo, thi + 1, x) : -1;
            hasLead = occ && j <= thi;
            hasFt = occ && j - 1 >= tlo;
            jl = j;
            if (hasLead) { xl = in.x[j]; vl = in.v[j]; tyl = in.ty[j]; }
            if (hasFt) { xFt = in.x[j - 1]; vFt = in.v[j - 1]; tyFt = in.ty[j - 1]; }
        }
        Lead Lt = {0, 0.0f, 0.0f, 0.0f, -1, 0.0f};
        if (hasLead) {
            Lt.kind = 1; Lt.xl = xl; Lt.vl = vl; Lt.ll = by_type(P.tlen, tyl); Lt.s = (xl - Lt.ll) - x;
            Lt.idx = jl;
        } else if (held) {
            Lt = stop_line_lead(len, x);
        } else if (nx >= 0) {
            if (!haveE2) {
                E2 = net.er[nx];
                haveE2 = true;
            }
            int nl2 = E2.lanes;
            int k2 = E2.lane_base + (lt < nl2 - 1 ? lt : nl2 - 1);
            int j2, tyr;
            float xr, vr;
            const bool ok = lane_rear(s.lanes, k2, ep, j2, xr, vr, tyr);
            const float ll = by_type(P.tlen, tyr);
            Lt.kind = ok ? 2 : 0;
            Lt.xl = ok ? xr : 0.0f;
            Lt.vl = ok ? vr : 0.0f;
            Lt.ll = ok ? ll : 0.0f;
            Lt.s = ok ? (len - x) + (xr - ll) : 0.0f;
            Lt.idx = ok ? j2 : -1;
        }
        if (!hasFt) { xFt = 0.0f; vFt = 0.0f; tyFt = 0; }
        // gap acceptance (Sec. 6.3.2)
        if (Lt.kind != 0 && Lt.s < P.s0) continue;
        if (hasFt && ((x - lme) - xFt) < P.s0) continue;
        int tfl = lead_flags(Lt);
        const float at = idm_acc_fl(P, A, Tg, kab, iv, v, Lt, tfl);
        if (at < -P.bsafe) continue;
        float dxt, vt;
        kin_move_fl(P, v, at, dxt, vt, tfl);
        clamp_to_leader_fl(Lt, dxt, vt, tfl);
        const float Xt = x + dxt;
        if (Xt >= len) continue;
        float an = 0.0f, ant = 0.0f;
        if (hasFt) {  // the lag follows with its own type's constants
            DrvRec Df = D;
            if (tyFt != ty) Df = net.drv[e * nt + tyFt];
            const float Af = Df.A, kf = Df.kab, ivf = Df.iv;
            an = idm_acc(P, Af, Tg, kf, ivf, vFt, relead(len, Lt, xFt));
            Lead Li = {1, (x - lme) - xFt, v, x, i, lme};
            ant = idm_acc(P, Af, Tg, kf, ivf, vFt, Li);
            if (ant < -P.bsafe) continue;
            Lead none = {0, 0.0f, 0.0f, 0.0f, -1, 0.0f};
            float afree = idm_acc(P, Af, Tg, kf, ivf, vFt, none);
            float dxF, vF2;
            kin_move(P, vFt, afree, dxF, vF2);
            if (((Xt - lme) - xFt) < dxF) continue;
        }
        float inc = 0.0f;
        if (!mand) {
            float d1 = at - ac;
            float d2 = hasFt ? (ant - an) : 0.0f;
            float d3 = 0.0f;
            if (hasF) {
                const float Af = Db.A, kf = Db.kab, ivf = Db.iv;
                Lead Lo = {1, (x - lme) - xF, v, x, i, lme};
                float ao = idm_acc(P, Af, Tg, kf, ivf, vF, Lo);
                float aot = idm_acc(P, Af, Tg, kf, ivf, vF, relead(len, L, xF));
                d3 = aot - ao;
            }
            inc = d1 + P.pol * (d2 + d3);
            if (!(inc > P.athr)) continue;
        }
        if (best < 0 || inc > best_inc) {
            best = lt; best_inc = inc; best_X = Xt; best_v = vt;
            best_fl = tfl; best_lead = Lt.idx;
        }
    }
    if (best >= 0) {
        if (kFull && tp.on) {
            tp.mode[i] = kModeChange;
            tp.cflags[i] = (unsigned short)best_fl;
            tp.clead[i] = best_lead;
        }
        stage_claim(CS, i, e, best, kChange, ty, best_X, best_v, 0.0f);
        return true;
    }
    return false;
}

// Departures (Sec. 6.2.2): a due trip enters the first link of its route in
// the lane with the most entry space, if that space holds its length plus s0,
// by claiming the entry cells; losers wait and try again every step.  Every
// trip of one queue (same first link, same type) sees the same lane and the
// same space, and all their claims cover cell 0 of that lane, so only the
// queue's head (its lowest vehicle id) can win, and its claim blocks every
// third claim any other member's would.  The head claims; the others are
// counted as claims that lost.
__device__ void decide_queue(const Params& P, const Net& net, const Trips& tr, const Scratch& s, unsigned ep,
                             unsigned long long tag, int t, int q, int& ghost, int& issued) {
    const int q0 = tr.qoff[q], qn = tr.qoff[q + 1] - q0;
    const int h = tr.qhead[q];
    int tl = tr.qtail[q];
    while (tl < qn && tr.qdep[q0 + tl] <= t) ++tl;  // release the trips due now
    tr.qtail[q] = tl;
    if (h == tl) return;  // nobody waiting
    const int e0 = tr.qedge[q];
    const int ty = tr.qtype[q];
    const EdgeRec E0 = net.er[e0];
    int best = -1;
    float bsp = 0.0f;
    for (int l = 0; l < E0.lanes; ++l) {
        int jl, tyr;
        float xr, vr;
        float sp = lane_rear(s.lanes, E0.lane_base + l, ep, jl, xr, vr, tyr) ? (xr - by_type(P.tlen, tyr)) : E0.len;
        if (best < 0 || sp > bsp) { best = l; bsp = sp; }
    }
    if (bsp >= by_type(P.tclaim, ty)) {
        int lo, hi;
        const ClaimRec C = net.cr[e0];
        claim_cells(P, C.ncell, ty, by_type(P.tlen, ty), lo, hi);
        push_claim(s, C, E0.lane_base, (q / kBlock) & (kSeg - 1), tag, tr.qvid[q0 + h], kInsert, -2 - q, e0, best,
                   by_type(P.tlen, ty),
                   0.0f, 1.0f, lo, hi);
        ghost += tl - h - 1;
        issued += tl - h;
    }
}

// The first qblocks blocks (a multiple of kSeg) take the departure queues, one
// thread per queue; the others the vehicles on the road in tiles of BS x R
// entries, R per thread: the step decision of every vehicle of a tile, then,
// for the vehicles it lists, the lane-change evaluation in the same thread.
// The two parts share nothing but the claim list.  (BS, R) is a launch shape
// the autotuner picks; results do not depend on it.  With kFull false the
// event tape, the utilization sampler and intersection control are compiled
// out, for launches where none of them is on (the host picks): their code
// and the arguments it keeps in registers cost the plain step spills and
// instructions.
template <int BS, int R, bool kFull>
__device__ __forceinline__ void decide_body(const Params& P, const Net& net, const Trips& tr, const Veh& in,
                                            const Scratch& s, const Tape& tp, Counters* ctr, int qblocks, int bid,
                                            int nblk) {
    constexpr int kTile = BS * R;
    const int t = ctr->t;
    const int N = ctr->n;
    const unsigned ep = *s.epoch;
    const unsigned long long tag = epoch_tag(ep);
    if (bid < qblocks) {
        int ghost = 0, issued = 0;
        for (int q = bid * BS + threadIdx.x; q < tr.nq; q += qblocks * BS)
            decide_queue(P, net, tr, s, ep, tag, t, q, ghost, issued);
        const unsigned long long gw = wave_sum_u64((unsigned long long)ghost);
        const unsigned long long iw = wave_sum_u64((unsigned long long)issued);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            seg_stat(s, kStGhost, gw);
            seg_stat(s, kStLost, gw);
            seg_stat(s, kStDepClaims, iw);
        }
        return;
    }
    static_assert(BS >= 2 * kTileHalo, "one thread per halo entry");
    __shared__ Tile<kTile + 2 * kTileHalo, kTileHalo> T;
    __shared__ ClaimStage<2 * kTile> CS;
    // XCD-aware mapping: the vehicle blocks (a multiple of kSeg) of XCD q take
    // the q-th eighth of the sorted entries, tiles in order, so that the link
    // and lane records of neighbouring vehicles are shared in that XCD's L2;
    // q is also the segment of every claim they append
    const int vb = bid - qblocks;
    const int q = vb & (kSeg - 1);
    const int nch = (N + kTile - 1) / kTile;
    const int c_end = (int)(((long long)nch * (q + 1)) / kSeg);
    int clamps = 0, arrivals = 0, listed = 0, claims = 0;
    if (kFull && tp.on && vb == 0 && threadIdx.x == 0) *tp.n = N;
    // a block's first tile of the eighth is the one its index names (no
    // atomic: a block without one leaves at once); the tiles after the first
    // of every block are taken in order from a counter of the eighth, so that
    // a block that meets fast tiles takes more of them
    __shared__ int s_c;
    const int c_beg = (int)(((long long)nch * q) / kSeg);
    const int nbs = (nblk - qblocks) / kSeg;  // vehicle blocks of the eighth
    if (threadIdx.x == 0) CS.n = 0;
    for (int it = 0;; ++it) {
        __syncthreads();  // s_c is read
        if (threadIdx.x == 0)
            s_c = c_beg + (it == 0 ? vb / kSeg : nbs + atomicAdd(s.tcnt + q * kSegStride, 1));
        __syncthreads();
        const int c = s_c;
        if (c >= c_end) break;
        const int b0 = c * kTile;
        // the tile and the entries on either side into LDS; the rest of the
        // own entries into registers
        int e[R], nx[R], vid[R], lcs[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = b0 + r * BS + threadIdx.x;
            const int ts = r * BS + threadIdx.x + kTileHalo;
            e[r] = 0; nx[r] = -1; vid[r] = 0; lcs[r] = 0;
            if (i < N) {
                T.key[ts] = in.key[i];
                T.x[ts] = in.x[i];
                T.v[ts] = in.v[i];
                T.ty[ts] = in.ty[i];
                e[r] = in.edge[i];
                nx[r] = in.next[i];
                vid[r] = in.vid[i];
                lcs[r] = in.lc[i];
            } else {
                T.key[ts] = kKeyPast;
                T.x[ts] = 0.0f;
                T.v[ts] = 0.0f;
                T.ty[ts] = 0;
            }
        }
        if (threadIdx.x < 2 * kTileHalo) {  // slots [0, H) before the tile, [H + kTile, 2 H + kTile) after it
            const int h = threadIdx.x;
            const bool before = h < kTileHalo;
            const int j = before ? b0 - kTileHalo + h : b0 + kTile + (h - kTileHalo);
            const int ts = before ? h : kTile + h;
            const bool has = j >= 0 && j < N;
            T.key[ts] = has ? in.key[j] : (before ? -1 : kKeyPast);
            T.x[ts] = has ? in.x[j] : 0.0f;
            T.v[ts] = has ? in.v[j] : 0.0f;
            T.ty[ts] = has ? (int)in.ty[j] : 0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = b0 + r * BS + threadIdx.x;
            const int ts = r * BS + threadIdx.x + kTileHalo;
            if (i < N) {
                Own o;
                if (decide_vehicle<kFull>(P, net, tr, in, s, tp, T, CS, ts, N, t, ep, tag, i, e[r], nx[r], vid[r], lcs[r],
                                   clamps, arrivals, o)) {
                    listed += 1;
                    claims += change_vehicle<kFull>(P, net, in, s, tp, T, CS, ts, b0, ep, o) ? 1 : 0;
                }
            }
        }
        __syncthreads();  // every claim of the tile is staged
        if (CS.n > kTile) {  // room for the next tile's claims: issue what is staged
            issue_claims<BS>(P, net, in, s, CS, q, tag);
            __syncthreads();
            if (threadIdx.x == 0) CS.n = 0;
        }
    }
    if (CS.n > 0) issue_claims<BS>(P, net, in, s, CS, q, tag);
    if (vb == 0 && threadIdx.x == 0) s.stay[N] = 0;
    unsigned long long cw = wave_sum_u64((unsigned long long)clamps);
    unsigned long long aw = wave_sum_u64((unsigned long long)arrivals);
    unsigned long long lw = wave_sum_u64((unsigned long long)listed);
    unsigned long long mw = wave_sum_u64((unsigned long long)claims);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        seg_stat(s, kStClamps, cw);
        seg_stat(s, kStArrived, aw);
        seg_stat(s, kStLcEval, lw);
        seg_stat(s, kStLcClaims, mw);
    }
}

template <int BS, int R, bool kFull>
__global__ __launch_bounds__(BS) void k_decide(Params P, Net net, Trips tr, Veh in, Scratch s, Tape tp,
                                               Counters* ctr, int qblocks) {
    decide_body<BS, R, kFull>(P, net, tr, in, s, tp, ctr, qblocks, (int)blockIdx.x, (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// k_resolve
// ---------------------------------------------------------------------------
constexpr int kCellBatch = 8;

__device__ __forceinline__ void resolve_body(const Params& P, const Net& net, const Trips& tr, const Veh& in,
                                             const Scratch& s, const Tape& tp, Counters* ctr, int bid, int nblk) {
    const int t = ctr->t;
    const int seg = bid & (kSeg - 1);  // the grid is a multiple of kSeg
    const int M = s.ccnt[seg * kSegStride];
    const int nb = nblk / kSeg;
    const unsigned ep = *s.epoch;
    const unsigned long long tag = epoch_tag(ep);
    if (bid == 0 && threadIdx.x < kSeg) s.tcnt[threadIdx.x * kSegStride] = 0;  // k_decide is done with them
    if (bid == 0 && threadIdx.x == 0) {
        ctr->scan_tile = 0;
        ctr->epoch_next = ep + 1u;
    }
    int lost = 0, departed = 0;
    for (int j = (bid / kSeg) * kBlock + threadIdx.x; j < M; j += nb * kBlock) {
        const int ci = seg * s.cl_seg + j;
        // the claim's fields, then everything they point to, before any branch:
        // the target lane's index record and key block bounds (for the gap),
        // the claimed cells, the source vehicle's link and entry time
        const int vid = s.cl_vid[ci];
        const int key = s.cl_key[ci];
        const int clo = s.cl_lo[ci], chi = s.cl_hi[ci];
        const long long cb = s.cl_cell[ci];
        const int kind = s.cl_kind[ci];
        const int src = s.cl_src[ci];
        const float cX = s.cl_X[ci], cf = s.cl_f[ci];
        int lo, hi;
        const bool occ = lane_range(s.lanes, key, ep, lo, hi);
        const int kb0 = s.lblk[key >> kLaneBlkLog], kb1 = s.lblk[(key >> kLaneBlkLog) + 1];
        const int sx = src >= 0 ? src : 0;
        const int se = in.edge[sx], skin = tr.kin[vid];
        const float sphin = tr.phin[vid];
        const int rcu = tr.rcur[vid], rbg = tr.rbeg[vid], rend = tr.rend[vid];
        // ownership of every claimed cell, kCellBatch cells at a time with all
        // the loads of a batch issued before any is compared (a car's claim
        // covers 8 cells: one round trip, not one per cell).  The first batch
        // is read unconditionally, with the reads beyond the last cell (or of
        // a claim that covers none) kept on a valid cell of the lane and not
        // counted, so that its reads go out with the others above
        const unsigned long long* cell = s.cells + cb;
        const unsigned long long mine = tag | (unsigned)vid;
        bool win = true;
        int c0 = clo;
        do {
            unsigned long long w[kCellBatch];
#pragma unroll
            for (int q = 0; q < kCellBatch; ++q) {
                const int c = c0 + q <= chi ? c0 + q : chi;
                w[q] = cell[c > 0 ? c : 0];
            }
#pragma unroll
            for (int q = 0; q < kCellBatch; ++q) win &= c0 + q > chi || w[q] == mine;
            c0 += kCellBatch;
        } while (c0 <= chi);
        // a crossing's or departure's place in its route after the move (both
        // cursors read with the rest; the kind picks one), and the route's
        // link after it, read for every kind at an index kept inside the route
        // and kept for a crossing or a departure that has one
        const int rc = kind == kCross ? rcu + 1 : rbg;
        int rn = tr.route_edges[rc + 1 < rend ? rc + 1 : rend - 1];
        // the claim's gap in the sorted order: inside its lane's run if the
        // lane is occupied, else before the first entry of a later lane; found
        // for every claim, won or lost, so that the search overlaps the read
        // above.  The empty asm after it keeps that read in its place: the
        // compiler would otherwise move it, and the route end's read with it,
        // into a branch of their own
        const int p = occ ? lb_x(in.x, lo, hi + 1, cX) : lb_key(in.key, kb0, kb1, key);
        asm("" : "+v"(rn));
        const int nn = (kind != kChange && rc + 1 < rend) ? rn : -1;
        if (tp.on && src >= 0) {
            if (kind == kCross) tp.mode[src] = win ? kModeCross : kModeYield;
            else tp.mode[src] = win ? kModeChange : kModeStay;
        }
        if (win) {
            if (src >= 0) s.stay[src] = 0;
            // its place in its gap and its slot in the list of movers, whose
            // two atomics are waited for together
            const int slot = atomicAdd(&s.mcnt[p], 1);
            const int m = seg * s.cl_seg + wave_slot(s.mvcnt + seg * kSegStride);
            s.mv_claim[m] = ci;
            s.mv_src[m] = src;
            s.mv_vid[m] = vid;
            s.mv_rc[m] = rc;
            s.mv_nx[m] = nn;
            s.mv_p[m] = p;
            s.mv_slot[m] = slot;
            if (kind == kCross) {
                record_exit(P, s, se, skin, sphin, cf, t);
                if (net.ctrl) {  // reaching the next link frees a stop node
                    const int h = net.head[se];
                    if (s.holder[h] == vid) s.holder[h] = -1;
                }
            }
            if (kind == kInsert) {
                tr.depart_actual[vid] = t + 1;
                atomicAdd(tr.qhead + (-2 - src), 1);  // the queue's head has left (one winner per queue)
                departed += 1;
            }
        } else {
            lost += 1;  // a losing departure simply stays at its queue's head
        }
    }
    unsigned long long lw = wave_sum_u64((unsigned long long)lost);
    unsigned long long dw = wave_sum_u64((unsigned long long)departed);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        seg_stat(s, kStLost, lw);
        seg_stat(s, kStDeparted, dw);
    }
}

__global__ __launch_bounds__(kBlock) void k_resolve(Params P, Net net, Trips tr, Veh in, Scratch s, Tape tp,
                                                    Counters* ctr) {
    resolve_body(P, net, tr, in, s, tp, ctr, (int)blockIdx.x, (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// k_scan: exclusive scan of w[i] = stay[i] + mcnt[i], i in [0, N], single pass
// with decoupled look-back; tiles are handed out in order by an atomic counter
// so a tile only ever waits on tiles already being processed.  It writes, per
// entry, the new position of the entry (its exclusive prefix plus the movers
// placed before it, those of gap i), complemented (~) when the entry does not
// stay, so that the re-sort reads one word per entry: cscan[i] ^ (cscan[i] >> 31)
// is that position, and the gap's first position is it minus mcnt[i].
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

__device__ __forceinline__ void scan_body(const Scratch& s, Counters* ctr) {
    const int N = ctr->n;
    const int total = N + 1;
    const int ntiles = (total + kScanTile - 1) / kScanTile;
    const unsigned ep = (*s.epoch % 0x3FFFFFFFu) + 1u;
    const int lane = threadIdx.x & (kWave - 1);
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
        unsigned stays = 0;  // bit q: entry base + q stays
        int tsum = 0;
        if (base + kScanItems <= total) {
            // a whole run: 16-byte loads of the counts and of the stay flags
            // (stay[N] is 0)
            static_assert(kScanItems % 16 == 0 && kScanItems <= 32, "a run is whole 16-byte words of flags");
            const int4* m4 = reinterpret_cast<const int4*>(s.mcnt + base);
            unsigned sw[kScanItems / 4];
#pragma unroll
            for (int u = 0; u < kScanItems / 16; ++u) {
                const uint4 st = reinterpret_cast<const uint4*>(s.stay + base)[u];
                sw[4 * u] = st.x;
                sw[4 * u + 1] = st.y;
                sw[4 * u + 2] = st.z;
                sw[4 * u + 3] = st.w;
            }
#pragma unroll
            for (int h = 0; h < kScanItems / 4; ++h) {
                const int4 m = m4[h];
                const int mm[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int sy = (int)((sw[h] >> (8 * r)) & 0xFFu);
                    const int w = mm[r] + sy;
                    vals[4 * h + r] = w;
                    stays |= (unsigned)(sy != 0) << (4 * h + r);
                    tsum += w;
                }
            }
        } else {
            for (int q = 0; q < kScanItems; ++q) {
                int idx = base + q;
                int w = 0;
                if (idx < total) {
                    const int sy = idx < N ? (int)s.stay[idx] : 0;
                    w = s.mcnt[idx] + sy;
                    stays |= (unsigned)(sy != 0) << q;
                }
                vals[q] = w;
                tsum += w;
            }
        }
        int agg;
        int excl = block_excl_scan(tsum, agg);
        if (threadIdx.x < kWave) {
            // publish this tile's aggregate, then look back over up to 64
            // predecessors at a time: sum aggregates down to the nearest tile
            // that has published its inclusive prefix
            if (lane == 0)
                __hip_atomic_store(&s.tile_status[tile], pack_status(ep, tile == 0 ? kFlagP : kFlagA, agg),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int prefix = 0;
            int hi = tile - 1;  // nearest predecessor not yet summed
            while (hi >= 0) {
                const int j = hi - lane;
                unsigned long long flag = kFlagP;  // before tile 0: an inclusive prefix of 0
                int val = 0;
                if (j >= 0) {
                    unsigned long long st =
                        __hip_atomic_load(&s.tile_status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    flag = ((unsigned)(st >> 34) == ep) ? ((st >> 32) & 3ull) : 0ull;
                    val = (int)(unsigned)(st & 0xFFFFFFFFull);
                }
                const unsigned long long isP = __ballot(flag == kFlagP);
                const unsigned long long notready = __ballot(flag == 0ull);
                const int firstP = isP ? (__ffsll((long long)isP) - 1) : kWave;
                const unsigned long long need = firstP >= kWave - 1 ? ~0ull : ((2ull << firstP) - 1ull);
                if (notready & need) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;  // a predecessor this tile depends on is still running
                }
                int mine = lane <= firstP ? val : 0;
                for (int o = kWave / 2; o > 0; o >>= 1) mine += __shfl_xor(mine, o, kWave);
                prefix += mine;
                if (firstP < kWave) break;
                hi -= kWave;
            }
            if (lane == 0) {
                if (tile > 0)
                    __hip_atomic_store(&s.tile_status[tile], pack_status(ep, kFlagP, prefix + agg), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                s_prefix = prefix;
                if (tile == ntiles - 1) ctr->n_next = prefix + agg;
            }
        }
        __syncthreads();
        int run = s_prefix + excl;
        // entry q's position: the prefix before it plus its gap's movers
        // (w - stay), complemented unless it stays
        auto pos = [&](int q, int r) {
            const int sy = (int)((stays >> q) & 1u);
            const int j = r + vals[q] - sy;
            return sy ? j : ~j;
        };
        if (base + kScanItems <= total) {
            int4* c4 = reinterpret_cast<int4*>(s.cscan + base);
#pragma unroll
            for (int h = 0; h < kScanItems / 4; ++h) {
                int4 o;
                o.x = pos(4 * h, run);
                run += vals[4 * h];
                o.y = pos(4 * h + 1, run);
                run += vals[4 * h + 1];
                o.z = pos(4 * h + 2, run);
                run += vals[4 * h + 2];
                o.w = pos(4 * h + 3, run);
                run += vals[4 * h + 3];
                c4[h] = o;
            }
        } else {
            for (int q = 0; q < kScanItems; ++q) {
                int idx = base + q;
                if (idx < total) s.cscan[idx] = pos(q, run);
                run += vals[q];
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_scan(Scratch s, Counters* ctr) { scan_body(s, ctr); }

// ---------------------------------------------------------------------------
// k_scatter: survivors to their new slot; movers stage their sort keys
// ---------------------------------------------------------------------------
// (the grid is a multiple of kSeg: block b stages the movers of segment b % kSeg)
__device__ __forceinline__ void scatter_body(const Params& P, const Veh& in, const Veh& out, const Scratch& s,
                                             const Tape& tp, Counters* ctr, int bid, int nblk) {
    const int N = ctr->n;
    for (int i = bid * kBlock + threadIdx.x; i < N; i += nblk * kBlock) {
        // every field read before the branch (almost every entry stays)
        const int j = s.cscan[i];  // the new position, complemented unless it stays
        const bool st = j >= 0;
        const int key = in.key[i], edge = in.edge[i], next = in.next[i], lc = in.lc[i];
        const int vid = in.vid[i];
        const unsigned char ty = in.ty[i];
        const float xs = s.xs[i], vs = s.vs[i], v = in.v[i];
        float fu = in.fuel[i], co = in.co[i];
        if (!st) continue;
        if (tp.on) tp.next[i] = j;
        out.key[j] = key;
        out.x[j] = xs;
        out.v[j] = vs;
        out.edge[j] = edge;
        out.next[j] = next;
        out.lc[j] = lc;
        out.vid[j] = vid;
        out.ty[j] = ty;
        emissions(P, v, vs, fu, co);
        out.fuel[j] = fu;
        out.co[j] = co;
    }
    const int seg = bid & (kSeg - 1);
    const int M = s.mvcnt[seg * kSegStride];
    const int nb = nblk / kSeg;
    for (int j = (bid / kSeg) * kBlock + threadIdx.x; j < M; j += nb * kBlock) {
        const int m = seg * s.cl_seg + j;
        const int p = s.mv_p[m];
        const int ci = s.mv_claim[m];
        const int g = s.mcnt[p];
        const int cp = s.cscan[p];
        const int b = (cp ^ (cp >> 31)) - g;
        s.mv_g[m] = g;
        s.grp_key[b + s.mv_slot[m]] = s.cl_key[ci];
        s.grp_X[b + s.mv_slot[m]] = s.cl_X[ci];
    }
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_scatter(
    Params P, Veh in, Veh out, Scratch s, Tape tp, Counters* ctr) {
    scatter_body(P, in, out, s, tp, ctr, (int)blockIdx.x, (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// k_place: movers take their rank inside their gap
// ---------------------------------------------------------------------------
__device__ __forceinline__ void place_body(const Params& P, const Trips& tr, const Veh& in, const Veh& out,
                                           const Scratch& s, const Tape& tp, int lc_none, Counters* ctr, int bid,
                                           int nblk) {
    const int t = ctr->t;
    const int seg = bid & (kSeg - 1);  // the grid is a multiple of kSeg
    const int M = s.mvcnt[seg * kSegStride];
    const int nb = nblk / kSeg;
    for (int jm = (bid / kSeg) * kBlock + threadIdx.x; jm < M; jm += nb * kBlock) {
        const int m = seg * s.cl_seg + jm;
        // reads in two rounds, each issued before any branch: the mover's
        // record (written by k_resolve); its claim, gap, source vehicle and type
        const int ci = s.mv_claim[m];
        const int p = s.mv_p[m];
        const int g = s.mv_g[m];
        const int src = s.mv_src[m], vid = s.mv_vid[m], rc = s.mv_rc[m], nn = s.mv_nx[m];
        const int cp = s.cscan[p];
        const int key = s.cl_key[ci];
        const float X = s.cl_X[ci];
        const int kind = s.cl_kind[ci];
        const float cv = s.cl_v[ci];
        const int cedge = s.cl_tedge[ci];
        const float cf = s.cl_f[ci];
        const int sx = src >= 0 ? src : 0;
        const float sfu = in.fuel[sx], sco = in.co[sx], sv = in.v[sx];
        const int snext = in.next[sx], slc = in.lc[sx];
        const int vty = tr.vtype[vid];
        const int b = (cp ^ (cp >> 31)) - g;
        int r = 0;
        if (g > 1) {  // four members of the gap at a time, their reads issued together
            for (int q0 = 0; q0 < g; q0 += 4) {
                int kq[4];
                float xq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int at = b + (q0 + q < g ? q0 + q : g - 1);
                    kq[q] = s.grp_key[at];
                    xq[q] = s.grp_X[at];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q0 + q < g && (kq[q] < key || (kq[q] == key && xq[q] < X))) ++r;
            }
        }
        const int j = b + r;
        if (tp.on && src >= 0) tp.next[src] = j;
        out.key[j] = key;
        out.x[j] = X;
        out.v[j] = cv;
        out.edge[j] = cedge;
        out.vid[j] = vid;
        out.ty[j] = vty;
        if (src >= 0) {
            float fu = sfu, co = sco;
            emissions(P, sv, cv, fu, co);
            out.fuel[j] = fu;
            out.co[j] = co;
        } else {
            out.fuel[j] = 0.0f;
            out.co[j] = 0.0f;
        }
        if (kind == kChange) {  // same link: the trip state stays
            out.next[j] = snext;
            out.lc[j] = t;
        } else {  // a crossing enters the next link of its route, a departure the first
            out.next[j] = nn;
            out.lc[j] = kind == kCross ? slc : lc_none;
            tr.rcur[vid] = rc;
            tr.kin[vid] = t + 1;
            tr.phin[vid] = kind == kCross ? cf : 1.0f;
        }
        s.mcnt[p] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_place(Params P, Trips tr, Veh in, Veh out, Scratch s, Tape tp,
                                                  int lc_none, Counters* ctr) {
    place_body(P, tr, in, out, s, tp, lc_none, ctr, (int)blockIdx.x, (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// k_lanes: index the lanes of the new sorted arrays (first and last entry per
// lane, tagged with the next step's epoch).  With `finalize` it also commits
// the step: the kernels of the step are the only readers of the counters it
// advances, and they have all completed.  8 waves per SIMD (no spills).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lanes_body(const Params& P, const Net& net, const Veh& buf, const Scratch& s,
                                           Counters* ctr, int finalize, int bid, int nblk) {
    const int N = finalize ? ctr->n_next : ctr->n;
    const unsigned ep = finalize ? ctr->epoch_next : *s.epoch;
    const unsigned long long tag = epoch_tag(ep);
    // few vehicles on a large network: every lane block finds its first entry
    // by a binary search over the (short) sorted keys; otherwise each entry
    // writes the lane blocks that begin at it
    const bool sparse = N < (s.nlblk >> 5);
    if (sparse)
        for (int b = bid * kBlock + threadIdx.x; b <= s.nlblk; b += nblk * kBlock)
            s.lblk[b] = lb_key(buf.key, 0, N, b << kLaneBlkLog);
    for (int j = bid * kBlock + threadIdx.x; j <= N; j += nblk * kBlock) {
        // the entry and its neighbours' lanes, its type, position and speed,
        // all read at once first (at indices kept inside the arrays, whose
        // values are not used where the index was moved)
        const int jc = j < N ? j : (N > 0 ? N - 1 : 0);
        const int k = buf.key[jc];
        const int kp = buf.key[j > 0 ? j - 1 : 0];
        const int kn = buf.key[j + 1 < N ? j + 1 : jc];
        const int tyj = buf.ty[jc];
        const float xj = buf.x[jc], vj = buf.v[jc];
        // lane blocks from the one after entry j-1's to entry j's begin at j;
        // a long run of them (empty lanes) is written by the whole wave, so no
        // single thread serialises it
        const int b0 = sparse ? 1 : (j == 0 ? 0 : (kp >> kLaneBlkLog) + 1);
        const int b1 = sparse ? 0 : (j == N ? s.nlblk : (k >> kLaneBlkLog));
        const bool longrun = b1 - b0 >= kWave / 2;
        if (!longrun)
            for (int b = b0; b <= b1; ++b) s.lblk[b] = j;
        {
            const unsigned long long act = __ballot(1);
            unsigned long long lm = __ballot(longrun);
            const int lane = (int)__lane_id();
            const int rank = __popcll(act & ((1ull << lane) - 1ull)), nact = __popcll(act);
            while (lm) {
                const int src = __ffsll((long long)lm) - 1;
                lm &= lm - 1ull;
                const int rb0 = __shfl(b0, src, kWave), rb1 = __shfl(b1, src, kWave), rj = __shfl(j, src, kWave);
                for (int b = rb0 + rank; b <= rb1; b += nact) s.lblk[b] = rj;
            }
        }
        if (j == N) continue;
        if (net.ctrl) {  // waiting at the line of a free stop node: ask to be admitted next step
            const int e = buf.edge[j];
            const int h = net.head[e];
            if (net.ctrl[h] == 1 && buf.next[j] >= 0 && s.holder[h] == -1 && (net.len[e] - xj) <= P.stop_dist &&
                vj <= P.stop_speed)
                atomicMin(s.stop_req + h, tag | (unsigned)buf.vid[j]);
        }
        LaneIx* lx = s.lanes + k;
        if (j == 0 || kp != k) {  // the lane's rearmost entry: epoch and first entry, type, position and speed
            *reinterpret_cast<uint2*>(&lx->ep) = make_uint2(ep, (unsigned)j);
            lx->ty = tyj;
            *reinterpret_cast<float2*>(&lx->x) = make_float2(xj, vj);
        }
        if (j == N - 1 || kn != k) lx->hi = j;
    }
    if (finalize && bid == 0 && threadIdx.x < kWave) {
        // fold the per-XCD lines into the counters (lane q reads line q) and
        // clear them for the next step
        const int q = threadIdx.x;
        unsigned long long v[kStDeparted + 2] = {};
        if (q < kSeg) {
            unsigned long long* st = s.sstat + q * kStatStride;
            for (int w = 0; w <= kStDeparted; ++w) v[w] = st[w];
            v[kStDeparted + 1] = (unsigned long long)s.ccnt[q * kSegStride];
            for (int w = 0; w < kStatStride; ++w) st[w] = 0;
            s.ccnt[q * kSegStride] = 0;
            s.mvcnt[q * kSegStride] = 0;
        }
        for (int w = 0; w < kStDeparted + 2; ++w) v[w] = wave_sum_u64(v[w]);
        if (q == 0) {
            ctr->updates += (unsigned long long)ctr->n;
            // claims: those with an entry, and departures that lose for certain
            ctr->claims += v[kStDeparted + 1] + v[kStGhost];
            ctr->clamps += v[kStClamps];
            ctr->arrived += v[kStArrived];
            ctr->claims_lost += v[kStLost];
            ctr->claims_dep += v[kStDepClaims];
            ctr->departed += v[kStDeparted];
            ctr->lc_eval += v[kStLcEval];
            ctr->claims_lc += v[kStLcClaims];
            ctr->n = ctr->n_next;
            ctr->t = ctr->t + 1;
            *s.epoch = ep;
        }
    }
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_lanes(
    Params P, Net net, Veh buf, Scratch s, Counters* ctr, int finalize) {
    lanes_body(P, net, buf, s, ctr, finalize, (int)blockIdx.x, (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// The whole step in one persistent launch: the resident blocks (a
// cooperative launch guarantees they run together) take the phases in turn,
// each phase's blocks as virtual blocks in a loop, with a device-wide barrier
// between phases; several steps per launch.  Same phases, same virtual
// launch shapes, same results as the six launches.
// ---------------------------------------------------------------------------
struct GridSync {
    unsigned count;  // blocks arrived at the current barrier
    unsigned gen;    // barriers completed
    unsigned fail;   // set when a wait gave up (the launch's results are then void)
};

// Every block waits here until all nblocks have arrived.  Each block's
// arrival is a release (its writes reach memory past its XCD's L2) and its
// departure one acquire (stale lines of its XCD's L2 and its CU's L1
// dropped), so each phase sees the writes of the one before on every XCD; the
// wait itself polls relaxed.  A wait that outlasts spin_limit polls, or finds
// another block's wait given up, flags the failure; the caller then ends the
// launch (returns true), so a launch always ends.
__device__ __forceinline__ bool grid_sync(GridSync* g, unsigned nblocks, unsigned spin_limit) {
    __shared__ int failed;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(&g->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(&g->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            // every other block's release is in the count this block read
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
            __hip_atomic_store(&g->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&g->gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&g->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > spin_limit ||
                    __hip_atomic_load(&g->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    __hip_atomic_fetch_or(&g->fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
        }
        failed = __hip_atomic_load(&g->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    }
    __syncthreads();
    return failed != 0;
}

// nsteps steps from buffer `parity` (b[parity] holds the state); the virtual
// grids are those of the six launches: qb + g8 decide blocks, g8 blocks for
// the claim, mover and scatter phases, g blocks for the lane index, and the
// scan's tiles handed out to every resident block
template <int R>
__global__ __launch_bounds__(kBlock) void k_steps(Params P, Net net, Trips tr, Veh b0, Veh b1, Scratch s,
                                                  Counters* ctr, GridSync* gs, int nsteps, int parity, int qb, int g8,
                                                  int g, int lc_none, unsigned spin_limit) {
    const Tape off{};
    const unsigned nb = gridDim.x;
    for (int k = 0; k < nsteps; ++k) {
        const bool odd = ((parity + k) & 1) != 0;
        const Veh& in = odd ? b1 : b0;
        const Veh& out = odd ? b0 : b1;
        for (int vb = blockIdx.x; vb < qb + g8; vb += nb) decide_body<kBlock, R, true>(P, net, tr, in, s, off, ctr, qb, vb, qb + g8);
        if (grid_sync(gs, nb, spin_limit)) return;
        for (int vb = blockIdx.x; vb < g8; vb += nb) resolve_body(P, net, tr, in, s, off, ctr, vb, g8);
        if (grid_sync(gs, nb, spin_limit)) return;
        scan_body(s, ctr);
        if (grid_sync(gs, nb, spin_limit)) return;
        for (int vb = blockIdx.x; vb < g8; vb += nb) scatter_body(P, in, out, s, off, ctr, vb, g8);
        if (grid_sync(gs, nb, spin_limit)) return;
        for (int vb = blockIdx.x; vb < g8; vb += nb) place_body(P, tr, in, out, s, off, lc_none, ctr, vb, g8);
        if (grid_sync(gs, nb, spin_limit)) return;
        for (int vb = blockIdx.x; vb < g; vb += nb) lanes_body(P, net, out, s, ctr, 1, vb, g);
        if (grid_sync(gs, nb, spin_limit)) return;
    }
}

// a restored or replaced state is indexed under a fresh epoch, so that no entry
// left by the state before it (tagged with the old epoch) reads as current
__global__ void k_next_epoch(unsigned* epoch) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *epoch += 1u;
}

__global__ void k_fill_u64(unsigned long long* p, long long n, unsigned long long v) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = v;
}

}  // namespace tsim
