/*
 * Route generation for the synthetic scenarios: single-source shortest paths
 * on a CSR road graph and extraction of edge-list routes from the
 * predecessor tree.  Routes are simulator INPUTS (the paper's trip planning
 * hands every vehicle a precomputed path, Sec. 6.3.1); nothing here is part of
 * the simulated dynamics.
 *
 * Determinism: the heap orders by (distance, node id) and an equal-distance
 * path never replaces the first one recorded, so the tree is a pure function
 * of the graph and the weights.  Both the oracle and the HIP path receive the
 * same route arrays.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

typedef struct { double d; int32_t n; } hitem;

static int hless(const hitem* a, const hitem* b) {
    return a->d < b->d || (a->d == b->d && a->n < b->n);
}

static void hpush(hitem* h, int64_t* sz, hitem it) {
    int64_t i = (*sz)++;
    h[i] = it;
    while (i > 0) {
        int64_t p = (i - 1) >> 1;
        if (!hless(&h[i], &h[p])) break;
        hitem t = h[i]; h[i] = h[p]; h[p] = t; i = p;
    }
}

static hitem hpop(hitem* h, int64_t* sz) {
    hitem top = h[0];
    h[0] = h[--(*sz)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *sz && hless(&h[l], &h[m])) m = l;
        if (r < *sz && hless(&h[r], &h[m])) m = r;
        if (m == i) break;
        hitem t = h[i]; h[i] = h[m]; h[m] = t; i = m;
    }
    return top;
}

/* Dijkstra from src.  dist[n] (inf if unreachable), pred_edge[n] (-1 at src /
 * unreachable).  Optional early exit: stop once every node flagged in
 * `need` (length n, may be NULL) is settled; `nneed` is how many are flagged.
 * Returns 0, or -1 on allocation failure. */
int ts_dijkstra(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                const double* w, int32_t src, double* dist, int32_t* pred_edge,
                const uint8_t* need, int32_t nneed) {
    int64_t m = row_ptr[n];
    hitem* heap = (hitem*)malloc(sizeof(hitem) * (size_t)(m + 2));
    uint8_t* done = (uint8_t*)calloc((size_t)n, 1);
    if (!heap || !done) { free(heap); free(done); return -1; }
    for (int32_t i = 0; i < n; ++i) { dist[i] = INFINITY; pred_edge[i] = -1; }
    int64_t sz = 0;
    dist[src] = 0.0;
    hitem s0 = {0.0, src};
    hpush(heap, &sz, s0);
    int32_t left = nneed;
    while (sz > 0) {
        hitem it = hpop(heap, &sz);
        int32_t u = it.n;
        if (done[u]) continue;
        done[u] = 1;
        if (need && need[u]) { if (--left <= 0) break; }
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col_idx[e];
            double nd = it.d + w[e];
            if (nd < dist[v]) {
                dist[v] = nd;
                pred_edge[v] = e;
                hitem ni = {nd, v};
                hpush(heap, &sz, ni);
            }
        }
    }
    free(heap); free(done);
    return 0;
}

/* For each destination, the edge list of the tree path src -> dst.
 * Pass out_edges == NULL to get lengths only (written to out_len).
 * With out_edges, route k is written at out_edges[out_off[k] ...].
 * tail[e] is the tail node of edge e.  Returns 0, or -1 if a destination is
 * unreachable or equal to src (empty route). */
int ts_paths(int32_t src, const int32_t* pred_edge, const int32_t* tail,
             int32_t ndst, const int32_t* dst, int64_t* out_len,
             const int64_t* out_off, int32_t* out_edges) {
    for (int32_t k = 0; k < ndst; ++k) {
        int32_t v = dst[k];
        if (v == src) return -1;
        int64_t len = 0;
        int32_t u = v;
        while (u != src) {
            int32_t e = pred_edge[u];
            if (e < 0) return -1;
            ++len;
            u = tail[e];
        }
        if (out_len) out_len[k] = len;
        if (out_edges) {
            int64_t pos = out_off[k] + len;
            u = v;
            while (u != src) {
                int32_t e = pred_edge[u];
                out_edges[--pos] = e;
                u = tail[e];
            }
        }
    }
    return 0;
}
