/* Oracle of the route planning used by iterative re-routing (Sec. 6.3.1) --
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
 *
 * Edge weights are travel times in integer milliseconds (>= 1), so every path
 * length is an exact integer and the shortest distance to a node is unique.
 * The route to a node is then made unique by one rule: the last edge of the
 * route into node w is the lowest-numbered edge e = (u -> w) with
 * dist[u] + w_e == dist[w].  Following that edge back from the destination
 * repeats the rule at u, down to the origin.
 *
 * or_sssp: textbook Dijkstra with a binary heap (lazy deletion), then the
 * predecessor rule above applied to every edge in id order.
 */
#include <stdint.h>
#include <stdlib.h>

#define OR_INF INT64_MAX

typedef struct {
    int64_t d;
    int32_t v;
} hitem;

static void heap_push(hitem* h, int64_t* n, hitem x) {
    int64_t i = (*n)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= x.d) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = x;
}

static hitem heap_pop(hitem* h, int64_t* n) {
    hitem top = h[0];
    hitem last = h[--(*n)];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= *n) break;
        if (c + 1 < *n && h[c + 1].d < h[c].d) c += 1;
        if (h[c].d >= last.d) break;
        h[i] = h[c];
        i = c;
    }
    if (*n > 0) h[i] = last;
    return top;
}

/* dist[v] (OR_INF if unreachable) and pred[v] (edge id, -1 at the source and
 * at unreachable nodes) from src.  Returns 0, -1 on bad input, -2 on no memory. */
int or_sssp(int32_t nn, int32_t ne, const int32_t* row_ptr, const int32_t* col_idx, const int64_t* w,
            int32_t src, int64_t* dist, int32_t* pred) {
    if (nn <= 0 || src < 0 || src >= nn || row_ptr[nn] != ne) return -1;
    for (int32_t e = 0; e < ne; ++e)
        if (w[e] < 1) return -1;
    hitem* heap = (hitem*)malloc(sizeof(hitem) * ((size_t)ne + 1));
    if (!heap) return -2;
    for (int32_t v = 0; v < nn; ++v) {
        dist[v] = OR_INF;
        pred[v] = -1;
    }
    int64_t hn = 0;
    dist[src] = 0;
    hitem s0 = {0, src};
    heap_push(heap, &hn, s0);
    while (hn > 0) {
        hitem it = heap_pop(heap, &hn);
        if (it.d > dist[it.v]) continue; /* stale entry */
        for (int32_t e = row_ptr[it.v]; e < row_ptr[it.v + 1]; ++e) {
            int32_t x = col_idx[e];
            int64_t nd = it.d + w[e];
            if (nd < dist[x]) {
                dist[x] = nd;
                hitem y = {nd, x};
                heap_push(heap, &hn, y);
            }
        }
    }
    free(heap);
    /* predecessor rule: lowest tight edge id; edges are visited in id order */
    for (int32_t u = 0; u < nn; ++u) {
        if (dist[u] == OR_INF) continue;
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t x = col_idx[e];
            if (x == src || pred[x] >= 0) continue;
            if (dist[u] + w[e] == dist[x]) pred[x] = e;
        }
    }
    return 0;
}
