// Adjoint of the car-following dynamics (included once, by trafficsim.hip).
//
// With the discrete events of a forward window held fixed (tape), positions
// and speeds are smooth functions of the per-class IDM parameters (Sec. 6.3.2,
// car-following equation) and so are the crossing-interpolated link travel
// times (Sec. 6.4).  Walking the recorded steps backwards, every vehicle
// turns the adjoint of its state after the step into the adjoint of its state
// before it, adds the terms that belong to the vehicle it followed, and adds
// its share of dLoss/dtheta.  Terms for a vehicle ahead are summed exactly in
// 64-bit fixed point (scale chosen per step from the largest term), so the
// result does not depend on the order of the atomic additions.
#pragma once

#include "common.h"

namespace tsim {

struct AdjState {
    const float* L1x;  // adjoint of the state after the step, by entry at the next step
    const float* L1v;
    float* L0x;        // adjoint of the state before the step, by entry at this step
    float* L0v;
    float* cgx;        // term for the vehicle ahead, by entry at this step
    float* cgv;
    int* cl;           // entry index of that vehicle, or -1
    long long* accx;   // fixed-point sums of the terms received, by entry at this step
    long long* accv;
    unsigned* maxbits; // largest |term| of the step (float bits)
    double* scale;     // fixed-point scale of the step
    float* lp;         // adjoint of each vehicle's current entry fraction, by vehicle id
    const float* dLdT; // dLoss / d(mean travel time) per link
    const unsigned long long* cnt;  // traversals per link
    double* gpart;     // per-thread partial sums of dLoss/dtheta [threads][ncls*4]
    int ncls;
    const unsigned char* vtype;  // vehicle type by vehicle id
};

// reverse of one applied motion (see the forward in step_kernels.h)
__device__ void motion_rev(const Params& P, float A, float T, float kab, float iv, int fl, float len, float x,
                           float v, float xL, float vL, float lL, float gdx, float gvn, float gf, float& gx,
                           float& gv, float& gxL, float& gvL, float& ga, float& gT, float& gkab, float& giv) {
    const bool lead = fl & kFHasLead;
    float s = 0.0f;
    if (lead) s = (fl & kFVirtual) ? len - x : (fl & kFLeadCross) ? (len - x) + (xL - lL) : (xL - lL) - x;
    float r = v * iv;
    float r2 = r * r;
    float fr = 1.0f - r2 * r2;
    float ss = 0.0f, se = 1.0f, q = 0.0f, acc0;
    if (!lead) {
        acc0 = A * fr;
    } else {
        float dyn = v * T + (v * (v - vL)) * kab;
        ss = (fl & kFDynFloor) ? P.s0 : P.s0 + dyn;
        se = (fl & kFSFloor) ? P.s_eps : s;
        q = ss / se;
        acc0 = A * (fr - q * q);
    }
    const float acc = (fl & kFAccFloor) ? -P.b_max : acc0;
    float dx = (fl & kFStop) ? (v * v) / (-2.0f * acc) : v * P.dt + acc * P.h;
    if (fl & kFDxFloor) dx = 0.0f;
    if (fl & kFClamp) dx = (fl & kFClampZero) ? 0.0f : s;

    float gs = 0.0f;
    if (!(fl & kFFOne) && gf != 0.0f && dx > 0.0f) {  // f = (len - x) / dx
        gx += -gf / dx;
        gdx += -gf * (len - x) / (dx * dx);
    }
    if (fl & kFClamp) {
        if (!(fl & kFClampZero)) gs += gdx;
        gdx = 0.0f;
        if (fl & kFClampV) {
            gvL += gvn;
            gvn = 0.0f;
        }
    }
    if (fl & kFDxFloor) gdx = 0.0f;
    float gacc;
    if (fl & kFStop) {
        gv += gdx * (2.0f * v) / (-2.0f * acc);
        gacc = gdx * (v * v) / (2.0f * acc * acc);
    } else {
        gv += gdx * P.dt + gvn;
        gacc = gdx * P.h + gvn * P.dt;
    }
    const float gacc0 = (fl & kFAccFloor) ? 0.0f : gacc;
    const float gfr = gacc0 * A;
    if (!lead) {
        ga += gacc0 * fr;
    } else {
        ga += gacc0 * (fr - q * q);
        float gq = -2.0f * q * A * gacc0;
        float gss = gq / se;
        float gse = -gq * q / se;
        if (!(fl & kFSFloor)) gs += gse;
        if (!(fl & kFDynFloor)) {
            float dv = v - vL;
            gv += gss * (T + (dv + v) * kab);
            gvL += -gss * v * kab;
            gT += gss * v;
            gkab += gss * v * dv;
        }
    }
    gv += gfr * (-4.0f * r2 * r * iv);
    giv += gfr * (-4.0f * r2 * r * v);
    if (lead) {
        gx += -gs;
        gxL += gs;
    }
}

// One applied motion with every branch forced to the recorded one (fl): the
// same expressions, in the same order, as the step's IDM, ballistic update and
// clamp, so in float at the recorded parameters it reproduces the recorded
// motion bit for bit.  dx before the crossing shift, vn the new speed.
template <class R>
__device__ __forceinline__ void motion_frozen(const Params& P, R A, R T, R kab, R iv, int fl, R len, R x, R v, R xL,
                                              R vL, R lL, R& dx, R& vn) {
    const bool lead = fl & kFHasLead;
    const R s0 = (R)P.s0, dt = (R)P.dt, h = (R)P.h;
    R s = 0;
    if (lead) s = (fl & kFVirtual) ? len - x : (fl & kFLeadCross) ? (len - x) + (xL - lL) : (xL - lL) - x;
    const R r = v * iv;
    const R r2 = r * r;
    const R r4 = r2 * r2;
    const R fr = (R)1 - r4;
    R acc;
    if (!lead) {
        acc = A * fr;
    } else {
        const R dv = v - vL;
        const R dyn = v * T + (v * dv) * kab;
        const R ss = (fl & kFDynFloor) ? s0 + (R)0 : s0 + dyn;
        const R q = ss / ((fl & kFSFloor) ? (R)P.s_eps : s);
        acc = A * (fr - q * q);
    }
    if (fl & kFAccFloor) acc = -(R)P.b_max;
    if (fl & kFStop) {
        dx = (v * v) / ((R)-2 * acc);
        vn = 0;
    } else {
        dx = v * dt + acc * h;
        vn = v + acc * dt;
    }
    if (fl & kFDxFloor) dx = 0;
    if (fl & kFClamp) {
        dx = (fl & kFClampZero) ? (R)0 : s;
        if (fl & kFClampV) vn = vL;
    }
}

// Frozen-event replay of one recorded step at the parameters in net, in
// precision R: every entry moves as recorded (leader, lane, link, crossing,
// branches) from the replayed state (rx, rv by entry at this step) into ox,
// ov (by entry at the next step, pre-filled with the recorded next state,
// which stands for the vehicles that enter the road).  A completed traversal
// adds its fraction difference f - phin to its link's sum F; phin (by vehicle
// id) is the fraction of the vehicle's last link entry.
// The IDM constants of a replay in precision R: per (class, type) a and
// 1/(2 sqrt(ab)), per class T, per (link, type) 1/v0.
template <class R>
struct ReplayCon {
    const R* A;
    const R* T;
    const R* kab;
    const R* iv;
};

template <class R>
__global__ __launch_bounds__(kBlock) void k_replay(Params P, Net net, ReplayCon<R> K, Tape tp, const R* rx,
                                                   const R* rv, R* ox, R* ov, R* phin, double* F,
                                                   const unsigned char* vtype) {
    const int N = *tp.n;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
        const int mode = tp.mode[i];
        const int nxt = tp.next[i];
        const int e = tp.edge[i];
        const R len = (R)net.len[e];
        if (mode == kModeYield) {  // waits at the link end
            ox[nxt] = len;
            ov[nxt] = 0;
            continue;
        }
        const int vid = tp.vid[i];
        const int fl = mode == kModeChange ? tp.cflags[i] : tp.flags[i];
        const int lead = mode == kModeChange ? tp.clead[i] : tp.lead[i];
        const R x = rx[i], v = rv[i];
        const R xL = lead >= 0 ? rx[lead] : (R)0;
        const R vL = lead >= 0 ? rv[lead] : (R)0;
        const R lL = lead >= 0 ? (R)by_type(P.tlen, vtype[tp.vid[lead]]) : (R)0;
        const int c = net.cls[e];
        const int ty = vtype[vid], nt = P.nt;
        R dx, vn;
        motion_frozen<R>(P, K.A[c * nt + ty], K.T[c], K.kab[c * nt + ty], K.iv[e * nt + ty], fl, len, x, v, xL, vL,
                         lL, dx, vn);
        const R xs = x + dx;
        if (mode == kModeCross || mode == kModeArrive) {
            const R fq = (len - x) / dx;
            const R f = dx > (R)0 ? ((fl & kFFOne) ? (R)1 : fq) : (R)0;
            atomicAdd(F + e, (double)f - (double)phin[vid]);
            if (mode == kModeCross) {
                phin[vid] = f;
                ox[nxt] = xs - len;
                ov[nxt] = vn;
            }
        } else {
            ox[nxt] = xs;
            ov[nxt] = vn;
        }
    }
}

// replay start: the recorded state of the first step, and the entry fraction
// of every vehicle id (1 for a vehicle not on the road yet: a departure
// enters with fraction 1)
template <class R>
__global__ void k_replay_init(Tape tp, R* rx, R* rv, R* phin, long long cap) {
    const long long n = (long long)*tp.n;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < cap; i += (long long)gridDim.x * kBlock) {
        phin[i] = 1;
        if (i < n) {
            rx[i] = (R)tp.x[i];
            rv[i] = (R)tp.v[i];
        }
    }
}

// entry fractions of the vehicles on the road at the window start
template <class R>
__global__ void k_replay_phin(const Veh ck, const float* ckphin, const Counters* ckctr, R* phin) {
    const int n = ckctr->n;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int id = ck.vid[i];
        phin[id] = (R)ckphin[id];
    }
}

// the recorded state of a step (stands for the vehicles entering the road)
template <class R>
__global__ void k_replay_seed(Tape tp, R* ox, R* ov) {
    const int N = *tp.n;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
        ox[i] = (R)tp.x[i];
        ov[i] = (R)tp.v[i];
    }
}

// own adjoint of every entry, its term for the vehicle ahead, theta partials
__global__ __launch_bounds__(kBlock) void k_adj_own(Params P, Net net, Tape tp, AdjState a) {
    const int N = *tp.n;
    const int gtid = blockIdx.x * kBlock + threadIdx.x;
    double* gp = a.gpart + (size_t)gtid * a.ncls * 4;
    float mx = 0.0f;
    for (int i = gtid; i < N; i += gridDim.x * kBlock) {
        const int mode = tp.mode[i];
        float gx = 0.0f, gv = 0.0f, gxL = 0.0f, gvL = 0.0f;
        int lead = -1;
        if (mode != kModeYield) {  // a vehicle waiting at the link end has a fixed outcome
            const int vid = tp.vid[i];
            const int e = tp.edge[i];
            const int nxt = tp.next[i];
            const float gxp = (mode != kModeArrive && nxt >= 0) ? a.L1x[nxt] : 0.0f;
            const float gvp = (mode != kModeArrive && nxt >= 0) ? a.L1v[nxt] : 0.0f;
            float gf = 0.0f;
            if (mode == kModeCross || mode == kModeArrive) {
                // traversal time dt*((t+1-kin) + f - phin): d/df = dt, d/dphin = -dt
                const float gtk = a.dLdT[e] / (float)a.cnt[e];
                gf = P.dt * gtk + (mode == kModeCross ? a.lp[vid] : 0.0f);
                a.lp[vid] = -P.dt * gtk;
            }
            const int fl = mode == kModeChange ? tp.cflags[i] : tp.flags[i];
            lead = mode == kModeChange ? tp.clead[i] : tp.lead[i];
            const float xL = lead >= 0 ? tp.x[lead] : 0.0f;
            const float vL = lead >= 0 ? tp.v[lead] : 0.0f;
            const float lL = lead >= 0 ? by_type(P.tlen, a.vtype[tp.vid[lead]]) : 0.0f;
            const int c = net.cls[e];
            const int ty = a.vtype[vid], nt = P.nt;
            const float A = net.cA[c * nt + ty], T = net.cT[c], kab = net.cKab[c * nt + ty];
            const float iv = net.inv_v0[e * nt + ty];
            float ga = 0.0f, gT = 0.0f, gkab = 0.0f, giv = 0.0f;
            gx = gxp;  // x' = x + dx (- len)
            motion_rev(P, A, T, kab, iv, fl, net.len[e], tp.x[i], tp.v[i], xL, vL, lL, gxp, gvp, gf, gx, gv, gxL,
                       gvL, ga, gT, gkab, giv);
            // theta = (v0_scale, T, a, b): iv = 1/(v0_scale*speed), kab = 1/(2 sqrt(ab)); where the
            // vehicle's type caps the speed or the acceleration, that parameter drops out
            const double vs = net.cVs[c], aa = A, bb = net.cB[c];
            const bool capv = net.capV[e * nt + ty], capa = net.capA[c * nt + ty];
            if (!capv) gp[4 * c + 0] += (double)giv * (-(double)iv / vs);
            gp[4 * c + 1] += (double)gT;
            if (!capa) gp[4 * c + 2] += (double)ga + (double)gkab * (-(double)kab / (2.0 * aa));
            gp[4 * c + 3] += (double)gkab * (-(double)kab / (2.0 * bb));
            if (lead < 0) {
                gxL = 0.0f;
                gvL = 0.0f;
            }
        }
        a.L0x[i] = gx;
        a.L0v[i] = gv;
        a.cgx[i] = gxL;
        a.cgv[i] = gvL;
        a.cl[i] = lead;
        mx = fmaxf(mx, fmaxf(fabsf(gxL), fabsf(gvL)));
    }
    for (int o = kWave / 2; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && mx > 0.0f) atomicMax(a.maxbits, __float_as_uint(mx));
}

__device__ __forceinline__ double fixed_scale(unsigned maxbits) {
    float mx = __uint_as_float(maxbits);
    if (!(mx > 0.0f)) return 1.0;
    // 2^52 / 2^ceil(log2 mx): up to 1024 terms for one vehicle stay below 2^62
    return ldexp(1.0, 52 - (ilogbf(mx) + 1));
}

// terms for the vehicles ahead, summed in fixed point
__global__ __launch_bounds__(kBlock) void k_adj_lead(Tape tp, AdjState a) {
    const int N = *tp.n;
    const double sc = fixed_scale(*a.maxbits);
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.scale = sc;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
        const int l = a.cl[i];
        if (l < 0) continue;
        const long long qx = __double2ll_rn((double)a.cgx[i] * sc);
        const long long qv = __double2ll_rn((double)a.cgv[i] * sc);
        if (qx) atomicAdd((unsigned long long*)&a.accx[l], (unsigned long long)qx);
        if (qv) atomicAdd((unsigned long long*)&a.accv[l], (unsigned long long)qv);
    }
}

// adjoint of the state before the step = own part + received terms
__global__ __launch_bounds__(kBlock) void k_adj_sum(Tape tp, AdjState a) {
    const int N = *tp.n;
    const double sc = *a.scale;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
        a.L0x[i] += (float)((double)a.accx[i] / sc);
        a.L0v[i] += (float)((double)a.accv[i] / sc);
        a.accx[i] = 0;
        a.accv[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.maxbits = 0u;
}

// dLoss/dtheta = sum of the per-thread partials, in thread order
__global__ void k_adj_reduce(const double* gpart, int nthreads, int nvals, float* out, double* out64) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nvals) return;
    double s = 0.0;
    for (int t = 0; t < nthreads; ++t) s += gpart[(size_t)t * nvals + k];
    out[k] = (float)s;
    if (out64) out64[k] = s;
}

__global__ void k_zero_f32(float* p, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = 0.0f;
}

__global__ void k_zero_f64(double* p, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = 0.0;
}

__global__ void k_zero_i64(long long* p, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = 0;
}

}  // namespace tsim
