"""Brute-force FP64 implementation of the microsimulation step, for tiny inputs.

Test infrastructure only.  It is written independently of ``oracle.c``: it
keeps vehicles in a plain Python list, finds every neighbour by scanning all
vehicles (O(N^2)) and resolves claims by checking every pair, so that the C
oracle's sorted lanes, lane index arrays and grouped claim resolution are
checked against a structure-free version of the same rules.

Rules (one synchronous step, all decisions read state t):
  * IDM acceleration (Sec. 6.3.2, car-following equation) with the vehicle
    ahead in the lane, or the rearmost vehicle of the mapped lane of the next
    link of the route, else free road;
  * ballistic update over dt, never past the rear of the vehicle ahead;
  * crossing the link end moves to the next link of the route (Sec. 6.3.1) if
    the claim on the entry cells wins, else the vehicle waits at the link end;
    crossing the end of the last link is arrival;
  * lane changes (Sec. 6.3.2): mandatory towards the turn band within the
    mandatory distance, discretionary by the MOBIL incentive, both behind gap
    acceptance; the target cells are claimed;
  * insertion at the route's first link, lane with most entry space, by claim.
A claim wins iff no overlapping claim on the same lane has a lower vehicle id.
"""
from __future__ import annotations

import math

import numpy as np

LC_NONE = -(1 << 30)


def _f(x):
    return float(np.float32(x))


class Brute:
    def __init__(self, scen):
        net, p, d = scen["net"], scen["params"], scen["demand"]
        self.row_ptr = [int(a) for a in net["row_ptr"]]
        self.head = [int(a) for a in net["col_idx"]]
        self.lanes = [int(a) for a in net["lanes"]]
        self.len = [_f(a) for a in net["length"]]
        ne = len(self.head)
        cls = net.get("link_class")
        self.cls = [0] * ne if cls is None else [int(a) for a in cls]
        idm = np.asarray(p["idm"], np.float32)
        self.vscale = [float(r[0]) for r in idm]
        self.T = [float(r[1]) for r in idm]
        # vehicle types (Sec. 6.3.5): (length, acceleration cap, speed cap)
        vt = p.get("vehicle_types")
        self.types = ([(_f(p["veh_length"]), math.inf, math.inf)] if vt is None else
                      [(_f(r[0]), _f(r[1]), _f(r[2])) for r in np.asarray(vt, np.float32)])
        self.A = [[min(float(r[2]), ty[1]) for ty in self.types] for r in idm]
        self.kab = [[1.0 / (2.0 * math.sqrt(min(float(r[2]), ty[1]) * float(r[3]))) for ty in self.types]
                    for r in idm]
        self.inv_v0 = [[1.0 / min(self.vscale[self.cls[e]] * _f(net["speed"][e]), ty[2]) for ty in self.types]
                       for e in range(ne)]
        self.ncell = [int(math.floor(self.len[e])) + 1 for e in range(ne)]
        self.dt = _f(p["dt"])
        self.h = 0.5 * self.dt * self.dt
        self.lveh = _f(p["veh_length"])
        self.s0 = _f(p["s0"])
        self.claim_len = [ty[0] + self.s0 for ty in self.types]
        self.s_eps = _f(p["s_eps"])
        self.b_max = _f(p["b_max"])
        self.pol = _f(p["mobil_p"])
        self.athr = _f(p["mobil_athr"])
        self.bsafe = _f(p["mobil_bsafe"])
        self.dmand = _f(p["mand_dist"])
        self.cool = int(p["lc_cooldown"])
        self.dt_us = int(round(self.dt * 1e6))
        self.dt_us_f = self.dt * 1e6
        ctrl = net.get("node_control")
        self.ctrl = None if ctrl is None else [int(c) for c in ctrl]
        self.green = int(p.get("signal_green", 20))
        self.stop_dist = _f(p.get("stop_dist", 3.0))
        self.stop_speed = _f(p.get("stop_speed", 0.5))
        self.holder = {}
        dep = np.asarray(d["depart_step"], np.int64)
        order = np.lexsort((np.arange(dep.size), dep))
        rp = np.asarray(d["route_ptr"], np.int64)
        re = [int(a) for a in d["route_edges"]]
        tr = np.asarray(d["trip_route"], np.int64)
        ttype = d.get("trip_type")
        self.trips = []
        for vid, i in enumerate(order):
            r = int(tr[i])
            self.trips.append({"dep": int(dep[i]), "route": re[rp[r]:rp[r + 1]], "orig": int(i),
                               "ty": 0 if ttype is None else int(ttype[i])})
        self.t = 0
        self.active = []
        self.pending = []
        self.depart_actual = [-1] * len(self.trips)
        self.arrive_step = [-1] * len(self.trips)
        self.st_cnt = [0] * ne
        self.st_steps = [0] * ne
        self.st_us = [0] * ne
        self.updates = 0
        if d.get("init_x") is not None:
            for vid, tr_ in enumerate(self.trips):
                i = tr_["orig"]
                self.active.append(self._new(vid, int(d["init_lane"][i]) if d.get("init_lane") is not None else 0,
                                             _f(d["init_x"][i]),
                                             _f(d["init_v"][i]) if d.get("init_v") is not None else 0.0, 0, 1.0))
                self.depart_actual[vid] = 0

    # -- helpers ---------------------------------------------------------
    def _new(self, vid, lane, x, v, kin, phin):
        route = self.trips[vid]["route"]
        return {"vid": vid, "cur": 0, "edge": route[0], "lane": lane, "x": x, "v": v,
                "lc": LC_NONE, "kin": kin, "phin": phin, "ty": self.trips[vid]["ty"]}

    def _len(self, q):
        return self.types[q["ty"]][0]

    def _next(self, q):
        route = self.trips[q["vid"]]["route"]
        return route[q["cur"] + 1] if q["cur"] + 1 < len(route) else -1

    def _on(self, e, l):
        return [q for q in self.active if q["edge"] == e and q["lane"] == l]

    def _idm(self, e, v, lead, ty):
        c = self.cls[e]
        r = v * self.inv_v0[e][ty]
        fr = 1.0 - (r * r) * (r * r)
        if lead is None:
            acc = self.A[c][ty] * fr
        else:
            s, vl = lead
            dyn = v * self.T[c] + (v * (v - vl)) * self.kab[c][ty]
            q = (self.s0 + max(0.0, dyn)) / max(s, self.s_eps)
            acc = self.A[c][ty] * (fr - q * q)
        return max(acc, -self.b_max)

    def _move(self, v, acc):
        if v + acc * self.dt < 0.0:
            return max((v * v) / (-2.0 * acc), 0.0), 0.0
        return max(v * self.dt + acc * self.h, 0.0), v + acc * self.dt

    def _clamp(self, lead, dx, vn):
        if lead is not None and dx > lead[0]:
            return max(lead[0], 0.0), min(vn, lead[1]), 1
        return dx, vn, 0

    def _rearmost(self, e, l):
        on = self._on(e, l)
        return min(on, key=lambda q: (q["x"], q["vid"])) if on else None

    def _held(self, e, nxt, vid):
        """is the movement e -> nxt held at the end of e (stop sign, red signal)?"""
        if self.ctrl is None or nxt < 0:
            return False
        h = self.head[e]
        if self.ctrl[h] == 1:
            return self.holder.get(h, -1) != vid
        if self.ctrl[h] == 2:
            inbound = [f for f in range(len(self.head)) if self.head[f] == h]
            outs = range(self.row_ptr[h], self.row_ptr[h + 1])
            movements = [(i, o) for i in inbound for o in outs]
            return movements[(self.t // self.green) % len(movements)] != (e, nxt)
        return False

    def _ahead(self, e, l, x, nxt, held=False):
        """vehicle ahead at lane l of link e for position x: (kind, xl, vl)"""
        ahead = [q for q in self._on(e, l) if q["x"] > x]
        if ahead:
            q = min(ahead, key=lambda q: (q["x"], q["vid"]))
            return (1, q["x"], q["v"], self._len(q))
        if held:
            return (3, self.len[e], 0.0, 0.0)
        if nxt >= 0:
            q = self._rearmost(nxt, min(l, self.lanes[nxt] - 1))
            if q is not None:
                return (2, q["x"], q["v"], self._len(q))
        return None

    def _gap(self, e, ah, x):
        if ah is None:
            return None
        kind, xl, vl, ll = ah
        if kind == 3:
            return (self.len[e] - x, 0.0)
        s = (xl - ll) - x if kind == 1 else (self.len[e] - x) + (xl - ll)
        return (s, vl)

    def _cells(self, e, X, ty):
        return max(0, math.floor(X - self.claim_len[ty])), min(self.ncell[e] - 1, math.floor(X))

    # -- one step ----------------------------------------------------------
    def _decide(self, q):
        e, l, x, v, ty = q["edge"], q["lane"], q["x"], q["v"], q["ty"]
        lme = self._len(q)
        nxt = self._next(q)
        held = self._held(e, nxt, q["vid"])
        same = [w for w in self._on(e, l) if (w["x"], w["vid"]) > (x, q["vid"])]
        if same:
            w = min(same, key=lambda w: (w["x"], w["vid"]))
            own = (1, w["x"], w["v"], self._len(w))
        elif held:
            own = (3, self.len[e], 0.0, 0.0)
        elif nxt >= 0:
            w = self._rearmost(nxt, min(l, self.lanes[nxt] - 1))
            own = None if w is None else (2, w["x"], w["v"], self._len(w))
        else:
            own = None
        L = self._gap(e, own, x)
        ac = self._idm(e, v, L, ty)
        dx, vn = self._move(v, ac)
        dx, vn, clamped = self._clamp(L, dx, vn)
        xs = x + dx
        out = {"clamped": clamped}
        if xs > self.len[e]:  # the front passes the link end strictly
            f = min((self.len[e] - x) / dx, 1.0) if dx > 0.0 else 0.0
            if nxt < 0:
                out.update(kind="arrive", f=f)
                return out
            tl = min(l, self.lanes[nxt] - 1)
            X = xs - self.len[e]
            out.update(kind="cross", f=f, tedge=nxt, tlane=tl, X=X, vc=vn, xs=self.len[e], vs=0.0,
                       cells=self._cells(nxt, X, ty))
            return out
        out.update(kind="stay", xs=xs, vs=vn)
        n = self.lanes[e]
        if n < 2 or self.t - q["lc"] < self.cool or x < lme:
            return out
        if nxt >= 0:
            hn = self.head[e]
            m = self.row_ptr[hn + 1] - self.row_ptr[hn]
            j = nxt - self.row_ptr[hn]
            lo = (j * n) // m
            hi = max(lo, -(-((j + 1) * n) // m) - 1)
        else:
            lo, hi = 0, n - 1
        d = self.len[e] - x
        inband = lo <= l <= hi
        mand = (not inband) and d <= self.dmand
        if mand:
            cands = [l + 1 if l < lo else l - 1]
        else:
            cands = [s for s in (l - 1, l + 1)
                     if 0 <= s < n and not (inband and d <= self.dmand and not lo <= s <= hi)]
        behind = [w for w in self._on(e, l) if (w["x"], w["vid"]) < (x, q["vid"])]
        F = max(behind, key=lambda w: (w["x"], w["vid"])) if behind else None
        best = None
        for lt in cands:
            ah = self._ahead(e, lt, x, nxt, held)
            Lt = self._gap(e, ah, x)
            lag = [w for w in self._on(e, lt) if w["x"] <= x]
            Ft = max(lag, key=lambda w: (w["x"], w["vid"])) if lag else None
            if Lt is not None and Lt[0] < self.s0:
                continue
            if Ft is not None and (x - lme) - Ft["x"] < self.s0:
                continue
            at = self._idm(e, v, Lt, ty)
            if at < -self.bsafe:
                continue
            dxt, vt = self._move(v, at)
            dxt, vt, _ = self._clamp(Lt, dxt, vt)
            Xt = x + dxt
            if Xt >= self.len[e]:
                continue
            an = ant = 0.0
            if Ft is not None:
                tf = Ft["ty"]
                an = self._idm(e, Ft["v"], self._gap(e, ah, Ft["x"]), tf)
                ant = self._idm(e, Ft["v"], ((x - lme) - Ft["x"], v), tf)
                if ant < -self.bsafe:
                    continue
                dxF, _ = self._move(Ft["v"], self._idm(e, Ft["v"], None, tf))
                if (Xt - lme) - Ft["x"] < dxF:
                    continue
            inc = 0.0
            if not mand:
                d2 = (ant - an) if Ft is not None else 0.0
                d3 = 0.0
                if F is not None:
                    ao = self._idm(e, F["v"], ((x - lme) - F["x"], v), F["ty"])
                    aot = self._idm(e, F["v"], self._gap(e, own, F["x"]), F["ty"])
                    d3 = aot - ao
                inc = (at - ac) + self.pol * (d2 + d3)
                if not inc > self.athr:
                    continue
            if best is None or inc > best[0]:
                best = (inc, lt, Xt, vt)
        if best is not None:
            out.update(kind="change", tedge=e, tlane=best[1], X=best[2], vc=best[3],
                       cells=self._cells(e, best[2], ty))
        return out

    def _exit(self, q, f):
        ns = self.t + 1 - q["kin"]
        e = q["edge"]
        self.st_cnt[e] += 1
        self.st_steps[e] += ns
        self.st_us[e] += ns * self.dt_us + int(round((f - q["phin"]) * self.dt_us_f))

    def step(self, n=1):
        for _ in range(n):
            self._step()

    def _step(self):
        t = self.t
        if self.ctrl is not None:
            # a free stop node admits the lowest id waiting at its line
            waiting = {}
            for q in self.active:
                h = self.head[q["edge"]]
                if self.ctrl[h] != 1 or self._next(q) < 0 or self.holder.get(h, -1) >= 0:
                    continue
                if self.len[q["edge"]] - q["x"] <= self.stop_dist and q["v"] <= self.stop_speed:
                    waiting[h] = min(waiting.get(h, q["vid"]), q["vid"])
            self.holder.update(waiting)
        dec = [self._decide(q) for q in self.active]
        cands = list(self.pending) + [v for v, tr in enumerate(self.trips)
                                      if tr["dep"] == t and self.depart_actual[v] < 0]
        claims = []  # (edge, lane, lo, hi, vid, ref)
        for i, (q, d) in enumerate(zip(self.active, dec)):
            if d["kind"] in ("cross", "change"):
                claims.append((d["tedge"], d["tlane"], d["cells"][0], d["cells"][1], q["vid"], ("veh", i)))
        ins_lane = {}
        for v in cands:
            e0 = self.trips[v]["route"][0]
            best, bsp = -1, 0.0
            for l in range(self.lanes[e0]):
                r = self._rearmost(e0, l)
                sp = (r["x"] - self._len(r)) if r is not None else self.len[e0]
                if best < 0 or sp > bsp:
                    best, bsp = l, sp
            ty = self.trips[v]["ty"]
            if bsp >= self.claim_len[ty]:
                ins_lane[v] = best
                lo, hi = self._cells(e0, self.types[ty][0], ty)
                claims.append((e0, best, lo, hi, v, ("ins", v)))
        won = set()
        for a in claims:
            if all(not (b[0] == a[0] and b[1] == a[1] and b[4] < a[4] and b[2] <= a[3] and a[2] <= b[3])
                   for b in claims):
                won.add(a[5])
        new = []
        for i, (q, d) in enumerate(zip(self.active, dec)):
            q = dict(q)
            if d["kind"] == "arrive":
                self._exit(q, d["f"])
                self.arrive_step[q["vid"]] = t + 1
                continue
            if d["kind"] == "cross" and ("veh", i) in won:
                if self.holder.get(self.head[q["edge"]], -1) == q["vid"]:
                    self.holder[self.head[q["edge"]]] = -1
                self._exit(q, d["f"])
                q.update(cur=q["cur"] + 1, edge=d["tedge"], lane=d["tlane"], x=d["X"], v=d["vc"],
                         kin=t + 1, phin=d["f"])
            elif d["kind"] == "change" and ("veh", i) in won:
                q.update(lane=d["tlane"], x=d["X"], v=d["vc"], lc=t)
            else:
                q.update(x=d["xs"], v=d["vs"])
            new.append(q)
        pend = []
        for v in cands:
            if ("ins", v) in won:
                new.append(self._new(v, ins_lane[v], self.types[self.trips[v]["ty"]][0], 0.0, t + 1, 1.0))
                self.depart_actual[v] = t + 1
            else:
                pend.append(v)
        self.updates += len(self.active)
        self.pending = pend
        self.active = new
        self.t = t + 1

    def vehicles(self):
        qs = sorted(self.active, key=lambda q: q["vid"])
        return {
            "vid": np.array([q["vid"] for q in qs], np.int32),
            "edge": np.array([q["edge"] for q in qs], np.int32),
            "lane": np.array([q["lane"] for q in qs], np.int32),
            "cursor": np.array([q["cur"] for q in qs], np.int32),
            "lc": np.array([q["lc"] for q in qs], np.int32),
            "kin": np.array([q["kin"] for q in qs], np.int32),
            "x": np.array([q["x"] for q in qs], np.float64),
            "v": np.array([q["v"] for q in qs], np.float64),
            "phin": np.array([q["phin"] for q in qs], np.float64),
        }

    def edge_stats(self):
        return {"count": np.array(self.st_cnt, np.int64), "tt_steps": np.array(self.st_steps, np.int64),
                "tt_us": np.array(self.st_us, np.int64)}
