/*
 * CPU ORACLE, differentiation part -- test infrastructure only (FP64).
 *
 * Frozen-event replay of an event tape recorded by the oracle's forward step,
 * the link travel-time loss, and its gradient by plain reverse mode.
 *
 * With the discrete events of a forward run held fixed (which vehicle is on
 * which link and lane, who follows whom, when a link end is crossed, which
 * branch of every max/min/stop/clamp was taken), the positions and speeds are
 * a smooth function of the per-class car-following parameters
 * theta_c = (v0_scale, T, a, b) of the IDM (Sec. 6.3.2, car-following
 * equation), and so are the crossing-interpolated link travel times
 * (Sec. 6.4 outputs).  The replay re-evaluates the same formulas as the step,
 * in the same order, with each branch forced to the recorded one:
 *   s   = (xL - l) - x  (same link),  (len - x) + (xL - l)  (next link),  len - x  (stop line)
 *   r   = v / v0,  fr = 1 - r^4
 *   acc = a fr                     (free road)
 *       = a (fr - (ss/max(s, s_eps))^2),  ss = s0 + max(0, vT + v(v - vL)/(2 sqrt(ab)))
 *   acc = max(acc, -b_max)
 *   stop:  dx = v^2/(-2 acc), v' = 0;   else dx = v dt + acc dt^2/2, v' = v + acc dt
 *   clamp: dx = max(s, 0), v' = min(v', vL)
 *   crossing: x' = x + dx - len, fraction f = min((len - x)/dx, 1)
 *   traversal time T = dt ((t+1 - kin) + f - phin), phin = f of the entry crossing (1 if inserted)
 *   loss = mean over links with traversals of (mean T on the link - target)^2.
 * The reverse pass walks the tape backwards and applies the chain rule to each
 * of these expressions; a leader's adjoint collects the terms of all its
 * followers.  Pinned by central finite differences of the replay itself and by
 * the replay reproducing the FP64 forward trajectory exactly.
 *
 * at_tape_states: instead of replaying the positions and speeds, take each
 * vehicle's state before every step from the tape (as the recording forward
 * computed it) and linearize there; the loss and gradient are then those of
 * that forward's own trajectory, evaluated in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    TF_HAS_LEAD = 1, TF_LEAD_CROSS = 2, TF_DYN_FLOOR = 4, TF_S_FLOOR = 8, TF_ACC_FLOOR = 16,
    TF_STOP = 32, TF_DX_FLOOR = 64, TF_CLAMP = 128, TF_CLAMP_ZERO = 256, TF_CLAMP_V = 512, TF_F_ONE = 1024,
    TF_VIRTUAL = 2048 /* the vehicle ahead is the stop line of a held movement: s = len - x, speed 0 */
};
enum { TM_STAY = 0, TM_CHANGE = 1, TM_YIELD = 2, TM_ARRIVE = 3, TM_CROSS = 4, TM_APPEAR = 5 };

typedef struct {
    double dt, h, lveh, s0, s_eps, b_max;
} cst_t;

typedef struct {
    double a, T, kab, iv; /* per (link, vehicle type): class parameters and 1/v0 */
    int capa, capv;       /* the type's acceleration / speed cap replaces a / v0_scale */
} par_t;

/* one motion, forward: returns dx, vn (before the crossing shift) and f */
static void motion(const cst_t* K, const par_t* P, int fl, double len, double x, double v, double xL,
                   double vL, double lL, double* dxo, double* vno, double* fo) {
    double s = 0.0;
    if (fl & TF_HAS_LEAD)
        s = (fl & TF_VIRTUAL) ? len - x : (fl & TF_LEAD_CROSS) ? (len - x) + (xL - lL) : (xL - lL) - x;
    double r = v * P->iv;
    double r2 = r * r;
    double fr = 1.0 - r2 * r2;
    double acc;
    if (!(fl & TF_HAS_LEAD)) {
        acc = P->a * fr;
    } else {
        double dyn = v * P->T + (v * (v - vL)) * P->kab;
        double ss = (fl & TF_DYN_FLOOR) ? K->s0 : K->s0 + dyn;
        double se = (fl & TF_S_FLOOR) ? K->s_eps : s;
        double q = ss / se;
        acc = P->a * (fr - q * q);
    }
    if (fl & TF_ACC_FLOOR) acc = -K->b_max;
    double dx, vn;
    if (fl & TF_STOP) {
        dx = (v * v) / (-2.0 * acc);
        vn = 0.0;
    } else {
        dx = v * K->dt + acc * K->h;
        vn = v + acc * K->dt;
    }
    if (fl & TF_DX_FLOOR) dx = 0.0;
    if (fl & TF_CLAMP) {
        dx = (fl & TF_CLAMP_ZERO) ? 0.0 : s;
        if (fl & TF_CLAMP_V) vn = vL;
    }
    *dxo = dx;
    *vno = vn;
    *fo = (fl & TF_F_ONE) ? 1.0 : (dx > 0.0 ? (len - x) / dx : 0.0);
}

/* one motion, reverse: given adjoints of dx (gdx), vn (gvn) and f (gf),
 * accumulate adjoints of x, v, xL, vL and of (a, T, kab, iv). */
static void motion_rev(const cst_t* K, const par_t* P, int fl, double len, double x, double v, double xL,
                       double vL, double lL, double gdx, double gvn, double gf, double* gx, double* gv,
                       double* gxL, double* gvL, double* ga, double* gT, double* gkab, double* giv) {
    /* recompute the forward intermediates */
    double s = 0.0;
    if (fl & TF_HAS_LEAD)
        s = (fl & TF_VIRTUAL) ? len - x : (fl & TF_LEAD_CROSS) ? (len - x) + (xL - lL) : (xL - lL) - x;
    double r = v * P->iv;
    double r2 = r * r;
    double fr = 1.0 - r2 * r2;
    double dyn = 0.0, ss = 0.0, se = 1.0, q = 0.0, acc0;
    if (!(fl & TF_HAS_LEAD)) {
        acc0 = P->a * fr;
    } else {
        dyn = v * P->T + (v * (v - vL)) * P->kab;
        ss = (fl & TF_DYN_FLOOR) ? K->s0 : K->s0 + dyn;
        se = (fl & TF_S_FLOOR) ? K->s_eps : s;
        q = ss / se;
        acc0 = P->a * (fr - q * q);
    }
    double acc = (fl & TF_ACC_FLOOR) ? -K->b_max : acc0;
    double dx;
    if (fl & TF_STOP) dx = (v * v) / (-2.0 * acc);
    else dx = v * K->dt + acc * K->h;
    if (fl & TF_DX_FLOOR) dx = 0.0;
    double dxf = dx; /* dx after the floor, before the clamp */
    if (fl & TF_CLAMP) dx = (fl & TF_CLAMP_ZERO) ? 0.0 : s;

    double gs = 0.0;
    /* f = (len - x) / dx  (dx after the clamp) */
    if (!(fl & TF_F_ONE) && gf != 0.0 && dx > 0.0) {
        *gx += -gf / dx;
        gdx += -gf * (len - x) / (dx * dx);
    }
    /* clamp */
    if (fl & TF_CLAMP) {
        if (!(fl & TF_CLAMP_ZERO)) gs += gdx;
        gdx = 0.0;
        if (fl & TF_CLAMP_V) {
            *gvL += gvn;
            gvn = 0.0;
        }
    }
    (void)dxf;
    /* floor of dx */
    if (fl & TF_DX_FLOOR) gdx = 0.0;
    /* kinematics */
    double gacc = 0.0;
    if (fl & TF_STOP) {
        /* dx = v^2 / (-2 acc) ; vn = 0 */
        *gv += gdx * (2.0 * v) / (-2.0 * acc);
        gacc += gdx * (v * v) / (2.0 * acc * acc);
    } else {
        *gv += gdx * K->dt + gvn;
        gacc += gdx * K->h + gvn * K->dt;
    }
    double gacc0 = (fl & TF_ACC_FLOOR) ? 0.0 : gacc;
    /* IDM */
    double gfr = gacc0 * P->a;
    if (!(fl & TF_HAS_LEAD)) {
        *ga += gacc0 * fr;
    } else {
        *ga += gacc0 * (fr - q * q);
        double gq = -2.0 * q * P->a * gacc0;
        double gss = gq / se;
        double gse = -gq * q / se;
        if (!(fl & TF_S_FLOOR)) gs += gse;
        if (!(fl & TF_DYN_FLOOR)) {
            double gdyn = gss;
            double dv = v - vL;
            *gv += gdyn * (P->T + (dv + v) * P->kab);
            *gvL += -gdyn * v * P->kab;
            *gT += gdyn * v;
            *gkab += gdyn * v * dv;
        }
    }
    /* fr = 1 - (v iv)^4 */
    *gv += gfr * (-4.0 * r2 * r * P->iv);
    *giv += gfr * (-4.0 * r2 * r * v);
    /* gap */
    if (fl & TF_HAS_LEAD) {
        *gx += -gs;
        *gxL += gs;
    }
}

int adj_eval(int64_t nrec, const int32_t* step, const int32_t* vid, const int32_t* mode, const int32_t* lead,
             const int32_t* flags, const int32_t* edge, const double* x0, const double* v0, int32_t nveh,
             int32_t ne, const double* len, const double* speed, const int32_t* cls, int32_t ncls,
             const double* theta, const double* fp, const double* target, const uint8_t* mask, double* loss,
             double* grad, double* tbar, double* xfin, double* vfin, int32_t at_tape_states, int32_t nt,
             const double* types, const int32_t* vtype) {
    cst_t K;
    K.dt = fp[0];
    K.h = 0.5 * fp[0] * fp[0];
    K.lveh = fp[1];
    K.s0 = fp[2];
    K.s_eps = fp[3];
    K.b_max = fp[4];
    double* x = (double*)calloc(nveh + 1, sizeof(double));
    double* v = (double*)calloc(nveh + 1, sizeof(double));
    double* phin = (double*)calloc(nveh + 1, sizeof(double));
    int32_t* phsrc = (int32_t*)malloc(sizeof(int32_t) * (nveh + 1)); /* record whose f is phin, or -1 */
    int32_t* kin = (int32_t*)calloc(nveh + 1, sizeof(int32_t));
    int32_t* where = (int32_t*)malloc(sizeof(int32_t) * (nveh + 1)); /* vid -> record of the current step */
    double* rx = (double*)malloc(sizeof(double) * (nrec + 1));      /* pre-state of each motion record */
    double* rv = (double*)malloc(sizeof(double) * (nrec + 1));
    double* rf = (double*)calloc(nrec + 1, sizeof(double));
    int32_t* rlead = (int32_t*)malloc(sizeof(int32_t) * (nrec + 1)); /* record of the leader at that step */
    int32_t* rtrav = (int32_t*)malloc(sizeof(int32_t) * (nrec + 1)); /* traversal index exiting here */
    int32_t* rphs = (int32_t*)malloc(sizeof(int32_t) * (nrec + 1));  /* phin source for that traversal */
    double* nx = (double*)malloc(sizeof(double) * (nrec + 1));
    double* nv = (double*)malloc(sizeof(double) * (nrec + 1));
    int64_t ntrav = 0;
    int32_t* tr_edge = (int32_t*)malloc(sizeof(int32_t) * (nrec + 1));
    double* tr_T = (double*)malloc(sizeof(double) * (nrec + 1));
    for (int32_t i = 0; i < nveh; ++i) { where[i] = -1; phsrc[i] = -1; }

    /* per (link, type): a vehicle type (Sec. 6.3.5) caps a and v0 = v0_scale * speed */
    par_t* P = (par_t*)malloc(sizeof(par_t) * ((size_t)ne * nt + 1));
    for (int32_t e = 0; e < ne; ++e) {
        const double* th = theta + 4 * cls[e];
        for (int32_t k = 0; k < nt; ++k) {
            par_t* q = &P[(size_t)e * nt + k];
            const double amax = types[3 * k + 1], vmax = types[3 * k + 2], v0 = th[0] * speed[e];
            q->capa = !(th[2] < amax);
            q->capv = !(v0 < vmax);
            q->a = q->capa ? amax : th[2];
            q->T = th[1];
            q->kab = 1.0 / (2.0 * sqrt(q->a * th[3]));
            q->iv = 1.0 / (q->capv ? vmax : v0);
        }
    }
#define PAR(e, i) (&P[(size_t)(e) * nt + vtype[i]])
#define LLEN(k) (rlead[k] >= 0 ? types[3 * vtype[lead[k]]] : 0.0)

    /* ---------------- forward replay ---------------- */
    int64_t r = 0;
    while (r < nrec) {
        if (mode[r] == TM_APPEAR) {
            int32_t i = vid[r];
            x[i] = x0[r];
            v[i] = v0[r];
            phin[i] = 1.0;
            phsrc[i] = -1;
            kin[i] = step[r];
            rtrav[r] = -1;
            ++r;
            continue;
        }
        int64_t g0 = r, g1 = r;
        while (g1 < nrec && step[g1] == step[g0] && mode[g1] != TM_APPEAR) ++g1;
        for (int64_t k = g0; k < g1; ++k) where[vid[k]] = (int32_t)k;
        for (int64_t k = g0; k < g1; ++k) {
            int32_t i = vid[k];
            /* the state before the step: replayed, or as recorded by the forward */
            rx[k] = at_tape_states ? x0[k] : x[i];
            rv[k] = at_tape_states ? v0[k] : v[i];
            rlead[k] = ((flags[k] & TF_HAS_LEAD) && !(flags[k] & TF_VIRTUAL)) ? where[lead[k]] : -1;
            rtrav[k] = -1;
        }
        for (int64_t k = g0; k < g1; ++k) {
            int32_t i = vid[k], e = edge[k];
            if (mode[k] == TM_YIELD) {
                nx[k] = len[e];
                nv[k] = 0.0;
                continue;
            }
            double xL = 0.0, vL = 0.0;
            if (rlead[k] >= 0) { xL = rx[rlead[k]]; vL = rv[rlead[k]]; }
            double dx, vn, f;
            motion(&K, PAR(e, i), flags[k], len[e], rx[k], rv[k], xL, vL, LLEN(k), &dx, &vn, &f);
            nx[k] = rx[k] + dx;
            nv[k] = vn;
            if (mode[k] == TM_CROSS || mode[k] == TM_ARRIVE) {
                rf[k] = f;
                tr_edge[ntrav] = e;
                tr_T[ntrav] = K.dt * ((double)(step[k] + 1 - kin[i]) + f - phin[i]);
                rtrav[k] = (int32_t)ntrav;
                rphs[k] = phsrc[i];
                ++ntrav;
                if (mode[k] == TM_CROSS) nx[k] = (rx[k] + dx) - len[e];
            }
        }
        for (int64_t k = g0; k < g1; ++k) {
            int32_t i = vid[k];
            if (mode[k] == TM_ARRIVE) continue;
            x[i] = nx[k];
            v[i] = nv[k];
            if (mode[k] == TM_CROSS) {
                phin[i] = rf[k];
                phsrc[i] = (int32_t)k;
                kin[i] = step[k] + 1;
            }
        }
        r = g1;
    }
    if (xfin) memcpy(xfin, x, sizeof(double) * nveh);
    if (vfin) memcpy(vfin, v, sizeof(double) * nveh);

    /* ---------------- loss ---------------- */
    double* sumT = (double*)calloc(ne + 1, sizeof(double));
    int64_t* cnt = (int64_t*)calloc(ne + 1, sizeof(int64_t));
    for (int64_t k = 0; k < ntrav; ++k) {
        sumT[tr_edge[k]] += tr_T[k];
        cnt[tr_edge[k]] += 1;
    }
    int64_t nm = 0;
    for (int32_t e = 0; e < ne; ++e)
        if (mask[e] && cnt[e] > 0) ++nm;
    double L = 0.0;
    double* gT = (double*)calloc(ne + 1, sizeof(double)); /* dL/dT of one traversal on each link */
    for (int32_t e = 0; e < ne; ++e) {
        double m = cnt[e] ? sumT[e] / (double)cnt[e] : 0.0;
        if (tbar) tbar[e] = m;
        if (mask[e] && cnt[e] > 0) {
            double d = m - target[e];
            L += d * d;
            gT[e] = 2.0 * d / ((double)nm * (double)cnt[e]);
        }
    }
    L = nm ? L / (double)nm : 0.0;
    *loss = L;

    /* ---------------- reverse pass ---------------- */
    if (grad) {
        memset(grad, 0, sizeof(double) * 4 * ncls);
        double* gx = (double*)calloc(nveh + 1, sizeof(double));
        double* gv = (double*)calloc(nveh + 1, sizeof(double));
        double* gfsrc = (double*)calloc(nrec + 1, sizeof(double)); /* adjoint of f at each crossing record */
        double* ngx = (double*)calloc(nrec + 1, sizeof(double));
        double* ngv = (double*)calloc(nrec + 1, sizeof(double));
        const size_t npar = (size_t)ne * nt + 1;
        double* ga = (double*)calloc(npar, sizeof(double));
        double* gTT = (double*)calloc(npar, sizeof(double));
        double* gkab = (double*)calloc(npar, sizeof(double));
        double* giv = (double*)calloc(npar, sizeof(double));
        /* traversal adjoints: dT/df = dt, dT/dphin = -dt */
        int64_t e1 = nrec;
        while (e1 > 0) {
            int64_t k1 = e1 - 1;
            if (mode[k1] == TM_APPEAR) {
                int32_t i = vid[k1];
                gx[i] = 0.0;
                gv[i] = 0.0;
                e1 = k1;
                continue;
            }
            int64_t g0 = k1;
            while (g0 > 0 && step[g0 - 1] == step[k1] && mode[g0 - 1] != TM_APPEAR) --g0;
            int64_t g1 = e1;
            for (int64_t k = g0; k < g1; ++k) { ngx[k] = 0.0; ngv[k] = 0.0; }
            for (int64_t k = g0; k < g1; ++k) {
                int32_t i = vid[k], e = edge[k];
                if (mode[k] == TM_YIELD) continue; /* constant outcome */
                double gxp = (mode[k] == TM_ARRIVE) ? 0.0 : gx[i];
                double gvp = (mode[k] == TM_ARRIVE) ? 0.0 : gv[i];
                double gf = 0.0;
                if (rtrav[k] >= 0) {
                    double gtk = gT[tr_edge[rtrav[k]]];
                    gf = K.dt * gtk + gfsrc[k];
                    if (rphs[k] >= 0) gfsrc[rphs[k]] += -K.dt * gtk;
                }
                double xL = 0.0, vL = 0.0;
                if (rlead[k] >= 0) { xL = rx[rlead[k]]; vL = rv[rlead[k]]; }
                double gxs = 0.0, gvs = 0.0, gxL = 0.0, gvL = 0.0;
                /* x' = x + dx (- len): both x and dx get gxp */
                gxs += gxp;
                const size_t pe = (size_t)e * nt + vtype[i];
                motion_rev(&K, &P[pe], flags[k], len[e], rx[k], rv[k], xL, vL, LLEN(k), gxp, gvp, gf, &gxs, &gvs,
                           &gxL, &gvL, &ga[pe], &gTT[pe], &gkab[pe], &giv[pe]);
                ngx[k] += gxs;
                ngv[k] += gvs;
                if (rlead[k] >= 0) {
                    ngx[rlead[k]] += gxL;
                    ngv[rlead[k]] += gvL;
                }
            }
            for (int64_t k = g0; k < g1; ++k) {
                int32_t i = vid[k];
                gx[i] = ngx[k];
                gv[i] = ngv[k];
            }
            e1 = g0;
        }
        /* chain to theta = (v0_scale, T, a, b) per class */
        for (int32_t e = 0; e < ne; ++e) {
            int32_t c = cls[e];
            const double* th = theta + 4 * c;
            for (int32_t k = 0; k < nt; ++k) {
                const size_t pe = (size_t)e * nt + k;
                double kab = P[pe].kab;
                if (!P[pe].capv) grad[4 * c + 0] += giv[pe] * (-P[pe].iv / th[0]);
                grad[4 * c + 1] += gTT[pe];
                if (!P[pe].capa) grad[4 * c + 2] += ga[pe] + gkab[pe] * (-kab / (2.0 * th[2]));
                grad[4 * c + 3] += gkab[pe] * (-kab / (2.0 * th[3]));
            }
        }
        free(gx); free(gv); free(gfsrc); free(ngx); free(ngv); free(ga); free(gTT); free(gkab); free(giv);
    }
    free(x); free(v); free(phin); free(phsrc); free(kin); free(where); free(rx); free(rv); free(rf);
    free(rlead); free(rtrav); free(rphs); free(nx); free(nv); free(tr_edge); free(tr_T); free(P);
    free(sumT); free(cnt); free(gT);
    return 0;
}
