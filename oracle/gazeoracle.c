/*
 * gazeoracle.c -- plain, slow CPU oracle for the gaze-line stereo graph cut
 * (Oguri & Shibata, "A new stereo formulation not using pixel and disparity
 * models").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source with the HIP library.
 *
 * What it computes, all in 64-bit integers:
 *   - the data-cost volume g(x, y, S) at every cross point   (Sec. 4.3, Sec. 3),
 *     grayscale truncated absolute difference or colour sum of absolute
 *     differences
 *   - the energy E(X) = sum_v g_v(X_v) + sum_(u,v) h~(X_u - X_v)  (Sec. 2, Sec. 3)
 *   - the layered (Ishikawa) graph as an explicit arc list    (Sec. 3, Fig. 4)
 *   - its exact max-flow by two unrelated textbook algorithms:
 *       Dinic (BFS level graph + blocking flow) and
 *       FIFO push-relabel with global relabelling (Sec. 4.4 cites this family)
 *   - the canonical labelling: the minimal source side of the minimum cut
 *   - brute-force enumeration of every labelling on tiny grids
 *   - exact scanline dynamic programming for one-row images
 *
 * Geometry (Sec. 3, Sec. 4.1).  A site is a gaze line (x, y), x in [0,w),
 * y in [0,h); a label is a depth number S in [0,m), S = 0 the front.  The
 * cross point (x, S, y) joins left pixel xl = x - S + (m-1) and right pixel
 * xr = x + S - (m-1) of row y, so disparity xl - xr = 2(m-1-S): one depth step
 * is two pixels of disparity (Sec. 4.1).  A cross point whose pixels fall
 * outside the image costs the truncation cap.
 *
 * Pairwise term (Sec. 3): h~(d) = h1*|d| + h2*(|d|-1)*T(|d|>1), h1 = penalty
 * (smoothness), h2 = inhibit (visibility).  It is convex (Sec. 2, eq. (1)),
 * so the energy is minimised exactly by one cut of the layered graph.
 *
 * Layered graph.  Per site v: nodes v_1..v_{m-1}, v_0 = s, v_m = t;
 * "v_k on the source side" means X_v >= k.
 *   chain     v_k -> v_{k+1}, cap g_v(k), k = 0..m-1  (cut iff X_v == k)
 *             reverse v_{k+1} -> v_k, cap INF for 1 <= k <= m-2
 *   level     u_k <-> v_k, cap h1 each way, k = 1..m-1
 *   diagonal  u_{k+1} -> v_k and v_{k+1} -> u_k, cap h2, k = 1..m-2
 * for every 4-neighbour pair (u, v) (Sec. 2), with per-direction (h1, h2).
 * The cut induced by X has capacity exactly E(X).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_NOMEM -2
#define ORC_E_PREFIX -3   /* a column was cut more than once */
#define ORC_E_TOO_BIG -4

/* Larger than any cut value this oracle is asked about. */
#define ORC_INF ((int64_t)1 << 52)

/* ------------------------------------------------------------------------ */
/* Data term: truncated absolute difference at each cross point.            */
/* ------------------------------------------------------------------------ */

/* cost[(S*h + y)*w + x] = min(|L(y, xl) - R(y, xr)|, cap), or cap when a
 * pixel lies outside the image. */
int orc_cost_volume(const uint8_t *left, const uint8_t *right, int w, int h,
                    int m, int cap, int32_t *cost)
{
    if (w < 0 || h < 0 || m < 1 || cap < 0 || !cost) return ORC_E_ARG;
    for (int S = 0; S < m; S++)
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                int xl = x - S + (m - 1);
                int xr = x + S - (m - 1);
                int32_t g = cap;
                if (xl >= 0 && xl < w && xr >= 0 && xr < w) {
                    int d = (int)left[y * w + xl] - (int)right[y * w + xr];
                    if (d < 0) d = -d;
                    g = d < cap ? d : cap;
                }
                cost[((int64_t)S * h + y) * w + x] = g;
            }
    return ORC_OK;
}

/* The colour data term of Sec. 4.3: the sum over the red, green and blue
 * channels of the absolute differences of the two pixels of the cross point
 * (0..765), capped at `cap` (cap >= 765 leaves it untruncated); a cross
 * point outside the image costs cap.  Images are [h][w][3] bytes, channels
 * interleaved. */
int orc_cost_volume_rgb(const uint8_t *left, const uint8_t *right, int w, int h,
                        int m, int cap, int32_t *cost)
{
    if (w < 0 || h < 0 || m < 1 || cap < 0 || !cost) return ORC_E_ARG;
    for (int S = 0; S < m; S++)
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                int xl = x - S + (m - 1);
                int xr = x + S - (m - 1);
                int32_t g = cap;
                if (xl >= 0 && xl < w && xr >= 0 && xr < w) {
                    int sad = 0;
                    for (int c = 0; c < 3; c++) {
                        int d = (int)left[((int64_t)y * w + xl) * 3 + c] -
                                (int)right[((int64_t)y * w + xr) * 3 + c];
                        sad += d < 0 ? -d : d;
                    }
                    g = sad < cap ? sad : cap;
                }
                cost[((int64_t)S * h + y) * w + x] = g;
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Energy, written out from its definition.                                  */
/* ------------------------------------------------------------------------ */

/* h~(d) = h1*|d| + h2*(|d|-1)*T(|d|>1)  (Sec. 3). */
static int64_t pair_term(int64_t h1, int64_t h2, int d)
{
    int a = d < 0 ? -d : d;
    return h1 * a + h2 * (int64_t)(a - 1) * (a > 1 ? 1 : 0);
}

int64_t orc_energy(const int32_t *cost, const int32_t *labels, int w, int h,
                   int m, int pen_h, int inh_h, int pen_v, int inh_v)
{
    int64_t e = 0;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            int S = labels[y * w + x];
            e += cost[((int64_t)S * h + y) * w + x];
        }
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            int S = labels[y * w + x];
            if (x + 1 < w) e += pair_term(pen_h, inh_h, S - labels[y * w + x + 1]);
            if (y + 1 < h) e += pair_term(pen_v, inh_v, S - labels[(y + 1) * w + x]);
        }
    (void)m;
    return e;
}

/* ------------------------------------------------------------------------ */
/* Explicit graph in compressed adjacency form.                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n;          /* nodes: 0 = s, 1 = t, then the grid nodes */
    int64_t narcs;
    int64_t *first;     /* n+1 offsets into the arc arrays */
    int32_t *head;      /* arc target */
    int64_t *rev;       /* index of the paired reverse arc */
    int64_t *res;       /* residual capacity */
    int64_t *cap0;      /* original capacity */
    int32_t *tail;      /* arc source (for checks) */
    int w, h, m;
    int32_t *lo, *hi;   /* optional per-site label windows (NULL: [0, m-1]) */
} orc_graph;

static int32_t node_id(int w, int h, int x, int y, int k)
{
    /* k in 1..m-1 */
    return 2 + (int32_t)((((int64_t)(k - 1) * h + y) * w) + x);
}

/* Map level k of site (x,y) to a node; k = 0 is s and k = m is t.  With a
 * label window [lo, hi] for the site, every level k <= lo is forced to the
 * source side (it is s) and every level k > hi to the sink side (it is t),
 * which restricts X_v to the window. */
static int32_t level_node(const orc_graph *g, int x, int y, int k)
{
    int lo = g->lo ? g->lo[y * g->w + x] : 0;
    int hi = g->hi ? g->hi[y * g->w + x] : g->m - 1;
    if (k <= lo) return 0;
    if (k > hi) return 1;
    return node_id(g->w, g->h, x, y, k);
}

typedef struct {
    orc_graph *g;
    int fill;           /* 0: count degrees, 1: place arcs */
    int64_t *pos;       /* next free slot per node (fill pass) */
} arc_sink;

static void add_pair(arc_sink *sk, int32_t a, int32_t b, int64_t cab, int64_t cba)
{
    orc_graph *g = sk->g;
    if (a == b) return;                 /* both ends forced to the same terminal */
    if (!sk->fill) {
        g->first[a + 1]++;
        g->first[b + 1]++;
        return;
    }
    int64_t ia = sk->pos[a]++;
    int64_t ib = sk->pos[b]++;
    g->head[ia] = b; g->tail[ia] = a; g->res[ia] = cab; g->cap0[ia] = cab; g->rev[ia] = ib;
    g->head[ib] = a; g->tail[ib] = b; g->res[ib] = cba; g->cap0[ib] = cba; g->rev[ib] = ia;
}

/* Emit every arc of the layered graph exactly once (as arc pairs). */
static void emit_arcs(arc_sink *sk, const int32_t *cost, int pen_h, int inh_h,
                      int pen_v, int inh_v)
{
    orc_graph *g = sk->g;
    int w = g->w, h = g->h, m = g->m;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            /* data chain: v_k -> v_{k+1} with cap g(k) */
            for (int k = 0; k < m; k++) {
                int64_t gk = cost[((int64_t)k * h + y) * w + x];
                int32_t a = level_node(g, x, y, k);
                int32_t b = level_node(g, x, y, k + 1);
                int64_t back = (k >= 1 && k <= m - 2) ? ORC_INF : 0;
                add_pair(sk, a, b, gk, back);
            }
        }
    for (int dir = 0; dir < 2; dir++) {
        int64_t h1 = dir == 0 ? pen_h : pen_v;
        int64_t h2 = dir == 0 ? inh_h : inh_v;
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                int ux = x, uy = y;
                int vx = dir == 0 ? x + 1 : x;
                int vy = dir == 0 ? y : y + 1;
                if (vx >= w || vy >= h) continue;
                /* same-level arcs u_k <-> v_k */
                for (int k = 1; k <= m - 1; k++)
                    add_pair(sk, level_node(g, ux, uy, k), level_node(g, vx, vy, k), h1, h1);
                /* diagonal arcs u_{k+1} -> v_k and v_{k+1} -> u_k */
                for (int k = 1; k <= m - 2; k++) {
                    add_pair(sk, level_node(g, ux, uy, k + 1), level_node(g, vx, vy, k), h2, 0);
                    add_pair(sk, level_node(g, vx, vy, k + 1), level_node(g, ux, uy, k), h2, 0);
                }
            }
    }
}

void orc_graph_free(orc_graph *g)
{
    if (!g) return;
    free(g->first); free(g->head); free(g->rev); free(g->res); free(g->cap0); free(g->tail);
    free(g->lo); free(g->hi);
    free(g);
}

/* Layered graph with optional per-site label windows lo[site] <= X <= hi[site]
 * (NULL for the unrestricted problem). */
orc_graph *orc_graph_build_window(const int32_t *cost, int w, int h, int m, int pen_h,
                                  int inh_h, int pen_v, int inh_v, const int32_t *lo,
                                  const int32_t *hi)
{
    if (w < 0 || h < 0 || m < 1) return NULL;
    if (pen_h < 0 || inh_h < 0 || pen_v < 0 || inh_v < 0) return NULL;
    int64_t nn = 2 + (int64_t)w * h * (m - 1);
    if (nn > INT32_MAX) return NULL;
    orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
    if (!g) return NULL;
    g->n = (int32_t)nn; g->w = w; g->h = h; g->m = m;
    if (lo && hi) {
        size_t ns = (size_t)w * h;
        g->lo = (int32_t *)malloc((ns ? ns : 1) * sizeof(int32_t));
        g->hi = (int32_t *)malloc((ns ? ns : 1) * sizeof(int32_t));
        if (!g->lo || !g->hi) { orc_graph_free(g); return NULL; }
        for (size_t i = 0; i < ns; i++) {
            if (lo[i] < 0 || hi[i] > m - 1 || lo[i] > hi[i]) { orc_graph_free(g); return NULL; }
            g->lo[i] = lo[i]; g->hi[i] = hi[i];
        }
    }
    g->first = (int64_t *)calloc((size_t)nn + 1, sizeof(int64_t));
    if (!g->first) { orc_graph_free(g); return NULL; }
    arc_sink sk = { g, 0, NULL };
    emit_arcs(&sk, cost, pen_h, inh_h, pen_v, inh_v);
    for (int64_t i = 0; i < nn; i++) g->first[i + 1] += g->first[i];
    g->narcs = g->first[nn];
    size_t na = (size_t)g->narcs > 0 ? (size_t)g->narcs : 1;
    g->head = (int32_t *)malloc(na * sizeof(int32_t));
    g->tail = (int32_t *)malloc(na * sizeof(int32_t));
    g->rev = (int64_t *)malloc(na * sizeof(int64_t));
    g->res = (int64_t *)malloc(na * sizeof(int64_t));
    g->cap0 = (int64_t *)malloc(na * sizeof(int64_t));
    sk.pos = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    if (!g->head || !g->tail || !g->rev || !g->res || !g->cap0 || !sk.pos) {
        free(sk.pos); orc_graph_free(g); return NULL;
    }
    memcpy(sk.pos, g->first, (size_t)nn * sizeof(int64_t));
    sk.fill = 1;
    emit_arcs(&sk, cost, pen_h, inh_h, pen_v, inh_v);
    free(sk.pos);
    return g;
}

orc_graph *orc_graph_build(const int32_t *cost, int w, int h, int m, int pen_h,
                           int inh_h, int pen_v, int inh_v)
{
    return orc_graph_build_window(cost, w, h, m, pen_h, inh_h, pen_v, inh_v, NULL, NULL);
}

int32_t orc_graph_nodes(const orc_graph *g) { return g->n; }
int64_t orc_graph_arcs(const orc_graph *g) { return g->narcs; }

/* Capacity of the cut induced by a labelling: source side = {s} and every
 * v_k with X_v >= k.  Used to check that the graph encodes E(X). */
int64_t orc_cut_capacity(const orc_graph *g, const int32_t *labels)
{
    int w = g->w, h = g->h;
    uint8_t *side = (uint8_t *)malloc((size_t)g->n);
    if (!side) return -1;
    side[0] = 1; side[1] = 0;
    for (int k = 1; k <= g->m - 1; k++)
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++)
                side[node_id(w, h, x, y, k)] = labels[y * w + x] >= k;
    int64_t c = 0;
    for (int64_t a = 0; a < g->narcs; a++)
        if (side[g->tail[a]] && !side[g->head[a]]) c += g->cap0[a];
    free(side);
    return c;
}

/* ------------------------------------------------------------------------ */
/* Residual reachability and label read-out.                                 */
/* ------------------------------------------------------------------------ */

/* Mark every node reachable by residual arcs from the seed set. */
static int reach_from(const orc_graph *g, uint8_t *mark)
{
    int32_t *queue = (int32_t *)malloc((size_t)g->n * sizeof(int32_t));
    if (!queue) return ORC_E_NOMEM;
    int64_t qh = 0, qt = 0;
    for (int32_t v = 0; v < g->n; v++)
        if (mark[v]) queue[qt++] = v;
    while (qh < qt) {
        int32_t u = queue[qh++];
        for (int64_t a = g->first[u]; a < g->first[u + 1]; a++) {
            int32_t v = g->head[a];
            if (g->res[a] > 0 && !mark[v]) { mark[v] = 1; queue[qt++] = v; }
        }
    }
    free(queue);
    return ORC_OK;
}

/* X_v = number of column nodes on the source side; the source side of a
 * column must be a prefix v_1..v_X (guaranteed by the INF reverse arcs). */
static int labels_from_side(const orc_graph *g, const uint8_t *side, int32_t *labels)
{
    int w = g->w, h = g->h, m = g->m;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            int X = 0, seen_out = 0;
            for (int k = 1; k <= m - 1; k++) {
                int in = side[level_node(g, x, y, k)];
                if (in) {
                    if (seen_out) return ORC_E_PREFIX;
                    X++;
                } else {
                    seen_out = 1;
                }
            }
            labels[y * w + x] = X;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Max-flow 1: Dinic.                                                        */
/* ------------------------------------------------------------------------ */

static int dinic_bfs(const orc_graph *g, int32_t *level, int32_t *queue)
{
    for (int32_t v = 0; v < g->n; v++) level[v] = -1;
    int64_t qh = 0, qt = 0;
    level[0] = 0; queue[qt++] = 0;
    while (qh < qt) {
        int32_t u = queue[qh++];
        for (int64_t a = g->first[u]; a < g->first[u + 1]; a++) {
            int32_t v = g->head[a];
            if (g->res[a] > 0 && level[v] < 0) { level[v] = level[u] + 1; queue[qt++] = v; }
        }
    }
    return level[1] >= 0;
}

/* Blocking flow with current-arc pointers and an explicit path stack. */
static int64_t dinic_block(orc_graph *g, const int32_t *level, int64_t *cur, int64_t *path)
{
    int64_t total = 0;
    int64_t depth = 0;              /* number of arcs on the path */
    int32_t u = 0;
    for (;;) {
        if (u == 1) {
            int64_t b = ORC_INF;
            for (int64_t i = 0; i < depth; i++) if (g->res[path[i]] < b) b = g->res[path[i]];
            for (int64_t i = 0; i < depth; i++) {
                g->res[path[i]] -= b;
                g->res[g->rev[path[i]]] += b;
            }
            total += b;
            /* retreat to the tail of the first saturated arc */
            int64_t cut = 0;
            while (cut < depth && g->res[path[cut]] > 0) cut++;
            depth = cut;
            u = depth == 0 ? 0 : g->head[path[depth - 1]];
            continue;
        }
        int advanced = 0;
        for (; cur[u] < g->first[u + 1]; cur[u]++) {
            int64_t a = cur[u];
            int32_t v = g->head[a];
            if (g->res[a] > 0 && level[v] == level[u] + 1) {
                path[depth++] = a;
                u = v;
                advanced = 1;
                break;
            }
        }
        if (advanced) continue;
        /* dead end: retreat */
        if (depth == 0) break;
        depth--;
        u = g->tail[path[depth]];
        cur[u]++;
    }
    return total;
}

int orc_maxflow_dinic(orc_graph *g, int64_t *flow_out)
{
    int32_t *level = (int32_t *)malloc((size_t)g->n * sizeof(int32_t));
    int32_t *queue = (int32_t *)malloc((size_t)g->n * sizeof(int32_t));
    int64_t *cur = (int64_t *)malloc((size_t)g->n * sizeof(int64_t));
    int64_t *path = (int64_t *)malloc((size_t)g->n * sizeof(int64_t));
    if (!level || !queue || !cur || !path) {
        free(level); free(queue); free(cur); free(path); return ORC_E_NOMEM;
    }
    int64_t flow = 0;
    while (dinic_bfs(g, level, queue)) {
        for (int32_t v = 0; v < g->n; v++) cur[v] = g->first[v];
        flow += dinic_block(g, level, cur, path);
    }
    free(level); free(queue); free(cur); free(path);
    *flow_out = flow;
    return ORC_OK;
}

/* Minimal source side after a max flow: residual reachability from s. */
int orc_labels_after_flow(const orc_graph *g, int32_t *labels)
{
    uint8_t *mark = (uint8_t *)calloc((size_t)g->n, 1);
    if (!mark) return ORC_E_NOMEM;
    mark[0] = 1;
    int rc = reach_from(g, mark);
    if (rc == ORC_OK) rc = labels_from_side(g, mark, labels);
    free(mark);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Max-flow 2: FIFO push-relabel with global relabelling (first phase only). */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t *excess;
    int32_t *height;
} orc_preflow;

/* Exact distance to t in the residual graph, by backward BFS; nodes that
 * cannot reach t get height n. */
static void global_relabel(const orc_graph *g, int32_t *height, int32_t *queue)
{
    int32_t n = g->n;
    for (int32_t v = 0; v < n; v++) height[v] = n;
    int64_t qh = 0, qt = 0;
    height[1] = 0; queue[qt++] = 1;
    while (qh < qt) {
        int32_t v = queue[qh++];
        for (int64_t a = g->first[v]; a < g->first[v + 1]; a++) {
            int32_t u = g->head[a];           /* arc v->u; its reverse u->v */
            if (u == 0) continue;
            if (height[u] == n && g->res[g->rev[a]] > 0) {
                height[u] = height[v] + 1;
                queue[qt++] = u;
            }
        }
    }
    height[0] = n;
}

int orc_maxflow_pushrelabel(orc_graph *g, int64_t *flow_out, int64_t *excess_out)
{
    int32_t n = g->n;
    int64_t *ex = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int32_t *ht = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *cur = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int32_t *fifo = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *bfsq = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    uint8_t *inq = (uint8_t *)calloc((size_t)n, 1);
    if (!ex || !ht || !cur || !fifo || !bfsq || !inq) {
        free(ex); free(ht); free(cur); free(fifo); free(bfsq); free(inq); return ORC_E_NOMEM;
    }
    /* saturate every arc out of s */
    for (int64_t a = g->first[0]; a < g->first[1]; a++) {
        int64_t c = g->res[a];
        if (c <= 0) continue;
        g->res[a] -= c; g->res[g->rev[a]] += c;
        ex[g->head[a]] += c; ex[0] -= c;
    }
    global_relabel(g, ht, bfsq);
    for (int32_t v = 0; v < n; v++) cur[v] = g->first[v];
    /* circular FIFO of active nodes (excess > 0, height < n, not s or t) */
    int64_t qh = 0, qn = 0;
    for (int32_t v = 2; v < n; v++)
        if (ex[v] > 0 && ht[v] < n) { fifo[(qh + qn) % n] = v; qn++; inq[v] = 1; }
    int64_t work = 0;
    const int64_t relabel_period = 6 * (int64_t)n + g->narcs / 2;
    while (qn > 0) {
        if (work > relabel_period) {
            work = 0;
            global_relabel(g, ht, bfsq);
            for (int32_t v = 0; v < n; v++) cur[v] = g->first[v];
            qh = 0; qn = 0;
            for (int32_t v = 2; v < n; v++) {
                inq[v] = 0;
                if (ex[v] > 0 && ht[v] < n) { fifo[qn++] = v; inq[v] = 1; }
            }
            continue;
        }
        int32_t u = fifo[qh]; qh = (qh + 1) % n; qn--; inq[u] = 0;
        /* discharge u */
        while (ex[u] > 0 && ht[u] < n) {
            if (cur[u] == g->first[u + 1]) {
                /* relabel: one above the lowest residual neighbour */
                int32_t hmin = n;
                for (int64_t a = g->first[u]; a < g->first[u + 1]; a++)
                    if (g->res[a] > 0 && ht[g->head[a]] < hmin) hmin = ht[g->head[a]];
                work += 12 + (g->first[u + 1] - g->first[u]);
                ht[u] = hmin + 1 < n ? hmin + 1 : n;
                cur[u] = g->first[u];
                continue;
            }
            int64_t a = cur[u];
            int32_t v = g->head[a];
            if (g->res[a] > 0 && ht[u] == ht[v] + 1) {
                int64_t d = ex[u] < g->res[a] ? ex[u] : g->res[a];
                g->res[a] -= d; g->res[g->rev[a]] += d;
                ex[u] -= d; ex[v] += d;
                if (v >= 2 && !inq[v] && ht[v] < n) {
                    fifo[(qh + qn) % n] = v; qn++; inq[v] = 1;
                }
                if (g->res[a] == 0) cur[u]++;
            } else {
                cur[u]++;
            }
        }
    }
    *flow_out = ex[1];
    if (excess_out) memcpy(excess_out, ex, (size_t)n * sizeof(int64_t));
    free(ex); free(ht); free(cur); free(fifo); free(bfsq); free(inq);
    return ORC_OK;
}

/* Minimal source side from a maximum preflow: residual reachability from s
 * and from every node that still holds positive excess.  Every such node is
 * on the source side of every minimum cut, and nothing reachable from it can
 * cross a saturated minimum cut, so this is the intersection of all minimum
 * source sides. */
int orc_labels_after_preflow(const orc_graph *g, const int64_t *excess, int32_t *labels)
{
    uint8_t *mark = (uint8_t *)calloc((size_t)g->n, 1);
    if (!mark) return ORC_E_NOMEM;
    mark[0] = 1;
    for (int32_t v = 2; v < g->n; v++) if (excess[v] > 0) mark[v] = 1;
    int rc = reach_from(g, mark);
    if (rc == ORC_OK && mark[1]) rc = ORC_E_ARG;    /* not a maximum preflow */
    if (rc == ORC_OK) rc = labels_from_side(g, mark, labels);
    free(mark);
    return rc;
}

/* Maximal source side: every node that cannot reach t in the residual graph.
 * Returns the labelling of the back-most optimal surface (diagnostics). */
int orc_labels_max_side(const orc_graph *g, int32_t *labels)
{
    /* backward reachability to t */
    int32_t n = g->n;
    uint8_t *to_t = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!to_t || !queue) { free(to_t); free(queue); return ORC_E_NOMEM; }
    int64_t qh = 0, qt = 0;
    to_t[1] = 1; queue[qt++] = 1;
    while (qh < qt) {
        int32_t v = queue[qh++];
        for (int64_t a = g->first[v]; a < g->first[v + 1]; a++) {
            int32_t u = g->head[a];
            if (!to_t[u] && g->res[g->rev[a]] > 0) { to_t[u] = 1; queue[qt++] = u; }
        }
    }
    for (int32_t v = 0; v < n; v++) to_t[v] = !to_t[v];
    int rc = labels_from_side(g, to_t, labels);
    free(to_t); free(queue);
    return rc;
}

/* Feasibility of the current flow: 0 <= flow <= cap on every arc pair and
 * conservation at every grid node (excess given, or zero when NULL). */
int orc_check_flow(const orc_graph *g, const int64_t *excess)
{
    int64_t *net = (int64_t *)calloc((size_t)g->n, sizeof(int64_t));
    if (!net) return ORC_E_NOMEM;
    for (int64_t a = 0; a < g->narcs; a++) {
        int64_t b = g->rev[a];
        if (g->rev[b] != a) { free(net); return 1; }
        /* flow on a = cap0(a) - res(a); paired arcs carry opposite flows */
        int64_t fa = g->cap0[a] - g->res[a];
        int64_t fb = g->cap0[b] - g->res[b];
        if (fa + fb != 0) { free(net); return 2; }
        if (g->res[a] < 0) { free(net); return 3; }
        if (fa > 0) { net[g->head[a]] += fa; net[g->tail[a]] -= fa; }
    }
    for (int32_t v = 2; v < g->n; v++) {
        int64_t want = excess ? excess[v] : 0;
        if (net[v] != want) { free(net); return 4; }
    }
    free(net);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One-call solve used by the tests and the CPU baseline.                   */
/* ------------------------------------------------------------------------ */

/* algo 0 = Dinic, 1 = push-relabel.  Writes the canonical labels, the
 * max-flow value and the energy of the labels. */
int orc_solve_window(const int32_t *cost, int w, int h, int m, int pen_h, int inh_h,
                     int pen_v, int inh_v, const int32_t *lo, const int32_t *hi, int algo,
                     int32_t *labels, int64_t *flow, int64_t *energy)
{
    if (m == 1) {
        for (int i = 0; i < w * h; i++) labels[i] = 0;
        *energy = orc_energy(cost, labels, w, h, m, pen_h, inh_h, pen_v, inh_v);
        *flow = *energy;
        return ORC_OK;
    }
    orc_graph *g = orc_graph_build_window(cost, w, h, m, pen_h, inh_h, pen_v, inh_v, lo, hi);
    if (!g) return ORC_E_NOMEM;
    int rc;
    if (algo == 0) {
        rc = orc_maxflow_dinic(g, flow);
        if (rc == ORC_OK) rc = orc_labels_after_flow(g, labels);
    } else {
        int64_t *ex = (int64_t *)malloc((size_t)g->n * sizeof(int64_t));
        if (!ex) { orc_graph_free(g); return ORC_E_NOMEM; }
        rc = orc_maxflow_pushrelabel(g, flow, ex);
        if (rc == ORC_OK) rc = orc_labels_after_preflow(g, ex, labels);
        free(ex);
    }
    orc_graph_free(g);
    if (rc == ORC_OK)
        *energy = orc_energy(cost, labels, w, h, m, pen_h, inh_h, pen_v, inh_v);
    return rc;
}

int orc_solve(const int32_t *cost, int w, int h, int m, int pen_h, int inh_h,
              int pen_v, int inh_v, int algo, int32_t *labels, int64_t *flow,
              int64_t *energy)
{
    return orc_solve_window(cost, w, h, m, pen_h, inh_h, pen_v, inh_v, NULL, NULL, algo,
                            labels, flow, energy);
}

/* ------------------------------------------------------------------------ */
/* Hierarchical approximation, level 1 (Sec. 4.5).                           */
/*                                                                          */
/* b x b x b neighbouring cross points form one delegate point: coarse site  */
/* (X, Y) = (x / b, y / b), coarse label Sc = S / b.  A first exact cut on   */
/* the delegate points picks, per coarse site, the label group holding the   */
/* surface; a second exact cut finds the real cross points inside a thin     */
/* skin around it: every fine site may only take the labels of its coarse    */
/* group and of the groups directly above and below.  Readings (the paper    */
/* omits the details): a delegate point costs the sum over its sites of the  */
/* cheapest label in its group; the coarse pairwise term keeps the fine      */
/* inhibit and scales the penalty by b^2 (a one-group step between coarse    */
/* sites is a b-level ramp over b rows of fine pairs).  b = 1 is the exact   */
/* minimisation.                                                             */
/* ------------------------------------------------------------------------ */

int orc_coarse_cost(const int32_t *cost, int w, int h, int m, int b, int32_t *coarse)
{
    if (b < 1 || w < 0 || h < 0 || m < 1) return ORC_E_ARG;
    int wc = (w + b - 1) / b, hc = (h + b - 1) / b, mc = (m + b - 1) / b;
    for (int Sc = 0; Sc < mc; Sc++)
        for (int Y = 0; Y < hc; Y++)
            for (int X = 0; X < wc; X++) {
                int64_t sum = 0;
                for (int y = Y * b; y < Y * b + b && y < h; y++)
                    for (int x = X * b; x < X * b + b && x < w; x++) {
                        int32_t best = INT32_MAX;
                        for (int S = Sc * b; S < Sc * b + b && S < m; S++) {
                            int32_t g = cost[((int64_t)S * h + y) * w + x];
                            if (g < best) best = g;
                        }
                        sum += best;
                    }
                coarse[((int64_t)Sc * hc + Y) * wc + X] = (int32_t)sum;
            }
    return ORC_OK;
}

/* Thin skin: labels of the coarse group and the groups above and below. */
int orc_skin_windows(const int32_t *coarse_labels, int w, int h, int m, int b, int32_t *lo,
                     int32_t *hi)
{
    if (b < 1) return ORC_E_ARG;
    int wc = (w + b - 1) / b;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            int Sc = coarse_labels[(y / b) * wc + x / b];
            int l = b * (Sc - 1), u = b * (Sc + 2) - 1;
            lo[y * w + x] = l < 0 ? 0 : l;
            hi[y * w + x] = u > m - 1 ? m - 1 : u;
        }
    return ORC_OK;
}

/* Level-1 approximation.  coarse_labels (optional) receives the first cut. */
int orc_approx_level1(const int32_t *cost, int w, int h, int m, int pen_h, int inh_h,
                      int pen_v, int inh_v, int b, int32_t *labels, int64_t *energy,
                      int32_t *coarse_labels)
{
    if (b < 1) return ORC_E_ARG;
    int wc = (w + b - 1) / b, hc = (h + b - 1) / b, mc = (m + b - 1) / b;
    size_t nc = (size_t)wc * hc;
    int32_t *cc = (int32_t *)malloc(((size_t)mc * nc + 1) * sizeof(int32_t));
    int32_t *cl = (int32_t *)malloc((nc + 1) * sizeof(int32_t));
    int32_t *lo = (int32_t *)malloc(((size_t)w * h + 1) * sizeof(int32_t));
    int32_t *hi = (int32_t *)malloc(((size_t)w * h + 1) * sizeof(int32_t));
    int rc = ORC_E_NOMEM;
    if (cc && cl && lo && hi) {
        int64_t f, e;
        rc = orc_coarse_cost(cost, w, h, m, b, cc);
        if (rc == ORC_OK)
            rc = orc_solve(cc, wc, hc, mc, b * b * pen_h, inh_h, b * b * pen_v, inh_v, 1, cl, &f, &e);
        if (rc == ORC_OK) rc = orc_skin_windows(cl, w, h, m, b, lo, hi);
        if (rc == ORC_OK)
            rc = orc_solve_window(cost, w, h, m, pen_h, inh_h, pen_v, inh_v, lo, hi, 1, labels,
                                  &f, energy);
        if (rc == ORC_OK && coarse_labels) memcpy(coarse_labels, cl, nc * sizeof(int32_t));
    }
    free(cc); free(cl); free(lo); free(hi);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Hierarchical approximation, level 2 (Sec. 4.5).                           */
/*                                                                          */
/* The wave-front pass runs over the whole thin skin and the push-relabel   */
/* loop cuts every block separately.  Readings (the paper omits the         */
/* details): the wave front is one pass down every column of the skin, from */
/* its top to its bottom, in which each free node hands the chain arc below  */
/* it as much of its excess as the arc's residual allows; a block is the     */
/* b x b sites of one delegate point over the full depth of their skin (all */
/* of them share one window), so only the arcs between delegate points go   */
/* unused; each block's cut is its exact minimum cut read off as the         */
/* minimal source side; a site's label is the deepest source-side node of   */
/* its column.  Splitting the skin's depth into b-level blocks as well would */
/* leave blocks in the middle of the skin without any sink.                  */
/*                                                                          */
/* State here is the skin with its terminals folded into node balances:     */
/* bal[v] = capacity of arcs into v from forced-source nodes (and s) minus   */
/* capacity of arcs from v to forced-sink nodes (and t); res[v][d] is the    */
/* residual of the arc from v to its neighbour in direction d, kept only    */
/* between two free nodes.                                                   */
/* ------------------------------------------------------------------------ */

/* neighbour offsets (dk, dy, dx) of the 14 arcs of a node v_k */
static const int NB[14][3] = {
    {+1, 0, 0}, {-1, 0, 0},                      /* chain down / up          */
    {0, 0, +1}, {0, 0, -1}, {0, +1, 0}, {0, -1, 0}, /* same level E W S N     */
    {-1, 0, +1}, {+1, 0, +1}, {-1, 0, -1}, {+1, 0, -1}, /* E/W one level up/down */
    {-1, +1, 0}, {+1, +1, 0}, {-1, -1, 0}, {+1, -1, 0}  /* S/N one level up/down */
};

/* Capacity of the arc from v_k (site x, y) to its neighbour in direction d
 * (Sec. 3, Fig. 4): chain down g(k), chain up unbounded, same level h1,
 * one level up (shallower) h2, one level down 0. */
static int64_t arc_cap(const int32_t *cost, int w, int h, int x, int y, int k, int d,
                       int pen_h, int inh_h, int pen_v, int inh_v)
{
    int dk = NB[d][0], dy = NB[d][1];
    if (d == 0) return cost[((int64_t)k * h + y) * w + x];
    if (d == 1) return ORC_INF;
    int horiz = dy == 0;
    if (dk == 0) return horiz ? pen_h : pen_v;
    if (dk < 0) return horiz ? inh_h : inh_v;
    return 0;
}

/* Tiny max-flow by shortest augmenting paths on a dense matrix. */
static int64_t ek_maxflow(int n, int64_t *cap, int src, int snk, uint8_t *src_side)
{
    int64_t flow = 0;
    int *prev = (int *)malloc(sizeof(int) * n), *q = (int *)malloc(sizeof(int) * n);
    for (;;) {
        for (int i = 0; i < n; i++) prev[i] = -1;
        int qh = 0, qt = 0;
        q[qt++] = src; prev[src] = src;
        while (qh < qt && prev[snk] < 0) {
            int u = q[qh++];
            for (int v = 0; v < n; v++)
                if (prev[v] < 0 && cap[(int64_t)u * n + v] > 0) { prev[v] = u; q[qt++] = v; }
        }
        if (prev[snk] < 0) break;
        int64_t b = ORC_INF;
        for (int v = snk; v != src; v = prev[v])
            if (cap[(int64_t)prev[v] * n + v] < b) b = cap[(int64_t)prev[v] * n + v];
        for (int v = snk; v != src; v = prev[v]) {
            cap[(int64_t)prev[v] * n + v] -= b;
            cap[(int64_t)v * n + prev[v]] += b;
        }
        flow += b;
    }
    /* minimal source side: reachable from src in the residual network */
    for (int i = 0; i < n; i++) src_side[i] = prev[i] >= 0;
    free(prev); free(q);
    return flow;
}

int orc_approx_level2(const int32_t *cost, int w, int h, int m, int pen_h, int inh_h,
                      int pen_v, int inh_v, int b, int32_t *labels, int64_t *energy,
                      int32_t *coarse_labels)
{
    if (b < 1 || m < 2) return ORC_E_ARG;
    int wc = (w + b - 1) / b, hc = (h + b - 1) / b, mc = (m + b - 1) / b;
    size_t ns = (size_t)w * h, nn = ns * (size_t)(m - 1);
    int32_t *cc = (int32_t *)malloc(((size_t)mc * wc * hc + 1) * sizeof(int32_t));
    int32_t *cl = (int32_t *)malloc(((size_t)wc * hc + 1) * sizeof(int32_t));
    int32_t *lo = (int32_t *)malloc((ns + 1) * sizeof(int32_t));
    int32_t *hi = (int32_t *)malloc((ns + 1) * sizeof(int32_t));
    int64_t *bal = (int64_t *)calloc(nn + 1, sizeof(int64_t));
    int64_t *res = (int64_t *)calloc(nn * 14 + 1, sizeof(int64_t));
    uint8_t *in_s = (uint8_t *)calloc(nn + 1, 1);
    int rc = ORC_E_NOMEM;
    if (!cc || !cl || !lo || !hi || !bal || !res || !in_s) goto done;
    {
        int64_t f, e;
        rc = orc_coarse_cost(cost, w, h, m, b, cc);
        if (rc == ORC_OK)
            rc = orc_solve(cc, wc, hc, mc, b * b * pen_h, inh_h, b * b * pen_v, inh_v, 1, cl, &f, &e);
        if (rc == ORC_OK) rc = orc_skin_windows(cl, w, h, m, b, lo, hi);
        if (rc != ORC_OK) goto done;
    }
#define NODE(x, y, k) ((((size_t)(k) - 1) * h + (y)) * w + (x))
#define FREE(x, y, k) ((k) > lo[(y) * w + (x)] && (k) <= hi[(y) * w + (x)])
    /* folded skin: balances and free-to-free residuals */
    for (int k = 1; k <= m - 1; k++)
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                if (!FREE(x, y, k)) continue;
                size_t v = NODE(x, y, k);
                for (int d = 0; d < 14; d++) {
                    int k2 = k + NB[d][0], y2 = y + NB[d][1], x2 = x + NB[d][2];
                    if (x2 < 0 || x2 >= w || y2 < 0 || y2 >= h) continue;
                    int lat = NB[d][1] != 0 || NB[d][2] != 0;
                    if (lat && (k2 < 1 || k2 > m - 1)) continue;     /* no lateral arc to s or t */
                    int64_t cout = arc_cap(cost, w, h, x, y, k, d, pen_h, inh_h, pen_v, inh_v);
                    /* capacity of the arc back from the neighbour */
                    int64_t cin;
                    if (d == 0) cin = ORC_INF;
                    else if (d == 1) cin = cost[((int64_t)(k - 1) * h + y) * w + x];
                    else cin = arc_cap(cost, w, h, x2, y2, k2, d ^ ((d >= 2 && d <= 5) ? 1 : 0),
                                       pen_h, inh_h, pen_v, inh_v);
                    if (d >= 6) {
                        /* opposite of a diagonal: one level the other way */
                        int up = NB[d][0] < 0;
                        int horiz = NB[d][1] == 0;
                        cin = up ? 0 : (horiz ? inh_h : inh_v);
                    }
                    int src = k2 <= (k2 >= 1 && k2 <= m - 1 ? lo[y2 * w + x2] : 0) || k2 == 0;
                    int snk = k2 == m || (k2 >= 1 && k2 <= m - 1 && k2 > hi[y2 * w + x2]);
                    if (src) bal[v] += cin;
                    else if (snk) bal[v] -= cout;
                    else res[v * 14 + d] = cout;
                }
            }
    /* wave front: one pass down every column of the skin */
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++)
            for (int k = lo[y * w + x] + 1; k < hi[y * w + x]; k++) {
                size_t v = NODE(x, y, k), u = NODE(x, y, k + 1);
                int64_t d = bal[v] < res[v * 14 + 0] ? bal[v] : res[v * 14 + 0];
                if (d <= 0) continue;
                bal[v] -= d; bal[u] += d;
                res[v * 14 + 0] -= d;
                /* the reverse (upward) arc is unbounded either way */
            }
    /* every block on its own */
    {
        int cap_nodes = b * b * (m - 1) + 2;
        int64_t *C = (int64_t *)malloc(sizeof(int64_t) * cap_nodes * cap_nodes);
        uint8_t *side = (uint8_t *)malloc(cap_nodes);
        size_t *ids = (size_t *)malloc(sizeof(size_t) * cap_nodes);
        int *kx = (int *)malloc(sizeof(int) * cap_nodes * 3);
        if (!C || !side || !ids || !kx) { free(C); free(side); free(ids); free(kx); rc = ORC_E_NOMEM; goto done; }
        for (int Y = 0; Y < hc; Y++)
            for (int X = 0; X < wc; X++) {
                int n = 0;
                for (int k = 1; k <= m - 1; k++)
                    for (int y = Y * b; y < Y * b + b && y < h; y++)
                        for (int x = X * b; x < X * b + b && x < w; x++)
                            if (FREE(x, y, k)) {
                                ids[n] = NODE(x, y, k);
                                kx[3 * n] = k; kx[3 * n + 1] = y; kx[3 * n + 2] = x;
                                n++;
                            }
                if (n == 0) continue;
                int N2 = n + 2, S = n, T = n + 1;
                memset(C, 0, sizeof(int64_t) * N2 * N2);
                for (int i = 0; i < n; i++) {
                    size_t v = ids[i];
                    if (bal[v] > 0) C[(int64_t)S * N2 + i] = bal[v];
                    if (bal[v] < 0) C[(int64_t)i * N2 + T] = -bal[v];
                    for (int d = 0; d < 14; d++) {
                        int k2 = kx[3 * i] + NB[d][0], y2 = kx[3 * i + 1] + NB[d][1],
                            x2 = kx[3 * i + 2] + NB[d][2];
                        for (int j2 = 0; j2 < n; j2++)
                            if (kx[3 * j2] == k2 && kx[3 * j2 + 1] == y2 && kx[3 * j2 + 2] == x2) {
                                int64_t r = d == 1 ? ORC_INF : res[v * 14 + d];
                                C[(int64_t)i * N2 + j2] += r;
                            }
                    }
                }
                ek_maxflow(N2, C, S, T, side);
                for (int i = 0; i < n; i++) in_s[ids[i]] = side[i];
            }
        free(C); free(side); free(ids); free(kx);
    }
    /* deepest source-side node of every column */
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            int X = lo[y * w + x];
            for (int k = lo[y * w + x] + 1; k <= hi[y * w + x]; k++)
                if (in_s[NODE(x, y, k)]) X = k;
            labels[y * w + x] = X;
        }
#undef NODE
#undef FREE
    *energy = orc_energy(cost, labels, w, h, m, pen_h, inh_h, pen_v, inh_v);
    if (coarse_labels) memcpy(coarse_labels, cl, (size_t)wc * hc * sizeof(int32_t));
    rc = ORC_OK;
done:
    free(cc); free(cl); free(lo); free(hi); free(bal); free(res); free(in_s);
    return rc;
}

/* Brute force restricted to per-site windows (tiny grids only). */
int orc_brute_force_window(const int32_t *cost, int w, int h, int m, int pen_h, int inh_h,
                           int pen_v, int inh_v, const int32_t *lo, const int32_t *hi,
                           int64_t *min_energy, int32_t *lo_labels)
{
    int n = w * h;
    double total = 1.0;
    for (int i = 0; i < n; i++) total *= (hi[i] - lo[i] + 1);
    if (total > 2.0e8) return ORC_E_TOO_BIG;
    int32_t *X = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!X) return ORC_E_NOMEM;
    for (int i = 0; i < n; i++) X[i] = lo[i];
    int64_t best = INT64_MAX;
    for (;;) {
        int64_t e = orc_energy(cost, X, w, h, m, pen_h, inh_h, pen_v, inh_v);
        if (e < best) {
            best = e;
            for (int i = 0; i < n; i++) lo_labels[i] = X[i];
        } else if (e == best) {
            for (int i = 0; i < n; i++) if (X[i] < lo_labels[i]) lo_labels[i] = X[i];
        }
        int i = 0;
        while (i < n && ++X[i] > hi[i]) { X[i] = lo[i]; i++; }
        if (i == n) break;
    }
    free(X);
    *min_energy = best;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Brute force over every labelling (tiny grids only).                       */
/* ------------------------------------------------------------------------ */

/* Enumerates all m^(w*h) labellings.  Returns the minimum energy, the number
 * of minimisers, and their pointwise minimum and maximum labellings. */
int orc_brute_force(const int32_t *cost, int w, int h, int m, int pen_h,
                    int inh_h, int pen_v, int inh_v, int64_t *min_energy,
                    int64_t *n_min, int32_t *lo_labels, int32_t *hi_labels)
{
    int n = w * h;
    double total = 1.0;
    for (int i = 0; i < n; i++) total *= m;
    if (total > 2.0e8) return ORC_E_TOO_BIG;
    int32_t *X = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    if (!X) return ORC_E_NOMEM;
    int64_t best = INT64_MAX, count = 0;
    for (;;) {
        int64_t e = orc_energy(cost, X, w, h, m, pen_h, inh_h, pen_v, inh_v);
        if (e < best) {
            best = e; count = 1;
            for (int i = 0; i < n; i++) lo_labels[i] = hi_labels[i] = X[i];
        } else if (e == best) {
            count++;
            for (int i = 0; i < n; i++) {
                if (X[i] < lo_labels[i]) lo_labels[i] = X[i];
                if (X[i] > hi_labels[i]) hi_labels[i] = X[i];
            }
        }
        int i = 0;
        while (i < n && ++X[i] == m) { X[i] = 0; i++; }
        if (i == n) break;
    }
    free(X);
    *min_energy = best;
    *n_min = count;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact dynamic programming along one row (h == 1), a textbook routine.     */
/* ------------------------------------------------------------------------ */

/* Forward and backward min-sum messages; label S is used by some minimiser
 * at x iff F_x(S) + B_x(S) - g_x(S) equals the minimum.  The canonical
 * (pointwise-minimum) labelling takes the smallest such S at every x. */
int orc_scanline_dp(const int32_t *cost, int w, int m, int pen, int inh,
                    int64_t *min_energy, int32_t *lo_labels)
{
    if (w <= 0) { *min_energy = 0; return ORC_OK; }
    int64_t *F = (int64_t *)malloc((size_t)w * m * sizeof(int64_t));
    int64_t *B = (int64_t *)malloc((size_t)w * m * sizeof(int64_t));
    if (!F || !B) { free(F); free(B); return ORC_E_NOMEM; }
#define G(x, S) ((int64_t)cost[(int64_t)(S) * w + (x)])
    for (int S = 0; S < m; S++) F[S] = G(0, S);
    for (int x = 1; x < w; x++)
        for (int S = 0; S < m; S++) {
            int64_t best = INT64_MAX;
            for (int P = 0; P < m; P++) {
                int64_t c = F[(x - 1) * m + P] + pair_term(pen, inh, P - S);
                if (c < best) best = c;
            }
            F[x * m + S] = best + G(x, S);
        }
    for (int S = 0; S < m; S++) B[(w - 1) * m + S] = G(w - 1, S);
    for (int x = w - 2; x >= 0; x--)
        for (int S = 0; S < m; S++) {
            int64_t best = INT64_MAX;
            for (int P = 0; P < m; P++) {
                int64_t c = B[(x + 1) * m + P] + pair_term(pen, inh, S - P);
                if (c < best) best = c;
            }
            B[x * m + S] = best + G(x, S);
        }
    int64_t emin = INT64_MAX;
    for (int S = 0; S < m; S++) if (F[(w - 1) * m + S] < emin) emin = F[(w - 1) * m + S];
    for (int x = 0; x < w; x++) {
        lo_labels[x] = -1;
        for (int S = 0; S < m; S++)
            if (F[x * m + S] + B[x * m + S] - G(x, S) == emin) { lo_labels[x] = S; break; }
    }
#undef G
    free(F); free(B);
    *min_energy = emin;
    return ORC_OK;
}
