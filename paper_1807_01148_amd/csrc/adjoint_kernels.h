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
