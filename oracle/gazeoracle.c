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

/* Moves delta units along arc a of the residual graph with no check at all
 * (tests use it to build infeasible flows for orc_check_flow). */
void orc_graph_push(orc_graph *g, int64_t a, int64_t delta)
{
    g->res[a] -= delta;
    g->res[g->rev[a]] += delta;
}

/* Index of the first arc from node u to node v, or -1. */
int64_t orc_graph_find_arc(const orc_graph *g, int32_t u, int32_t v)
{
    for (int64_t a = g->first[u]; a < g->first[u + 1]; a++)
        if (g->head[a] == v) return a;
    return -1;
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
/* The wave-front fetch runs over the whole thin skin, as in level 1, and   */
/* the push-relabel loop cuts every block (b x b x b cross points) on its    */
/* own.  The paper omits the details; the readings here are:                 */
/*   skin    the level-1 windows; levels outside them are folded into node   */
/*           balances, so the state is a preflow on the skin's free nodes    */
/*           with excess (positive balance) and deficits (negative);        */
/*   wave    the wave-front pre-phase of Sec. 4.4 (an initialisation, then  */
/*           A-1 wave steps): the initialisation gives every free node its   */
/*           exact residual distance to                                      */
/*           the nearest deficit (deficits at 1, unreachable at infinity);   */
/*           each of the A-1 wave steps is synchronous: every node with      */
/*           excess and finite height pushes, arc by arc in a fixed order,   */
/*           min(excess, residual) to neighbours exactly one lower (heights  */
/*           of the step's start), then every node that holds excess after   */
/*           the inflow is merged is lifted to one above its lowest residual */
/*           neighbour if that is higher (again the heights of the step's    */
/*           start: a Jacobi step, so the result does not depend on the      */
/*           order in which nodes are visited);                              */
/*   block   the free nodes of the b x b sites of one delegate point whose   */
/*           level k lies in the label group k / b (the node that carries    */
/*           the chain arc of label k); its push-relabel loop uses the arcs  */
/*           between its own nodes only and runs in rounds: exact in-block   */
/*           distances to the block's deficits, stop if no node with excess  */
/*           has a finite one, else 2n synchronous push / relabel steps of   */
/*           the rule above (n = nodes of the block);                       */
/*   cut     read off the final state as a push-relabel solver reads it      */
/*           from its distances: a free node is on the sink side iff a       */
/*           residual path leads from it to a node whose deficit is still    */
/*           unfilled (the maximal source side), and X_v counts the source- */
/*           side levels of the column (a prefix, through the unbounded      */
/*           upward chain arcs).                                             */
/* Once the state is a maximum preflow of the skin (a long enough wave, or   */
/* blocks that cover the skin) this is the back-most minimum of E inside the */
/* windows.                                                                  */
/* ------------------------------------------------------------------------ */

/* neighbour offsets (dk, dy, dx) of the 14 arcs of a node v_k */
static const int NB[14][3] = {
    {+1, 0, 0}, {-1, 0, 0},                      /* chain down / up          */
    {0, 0, +1}, {0, 0, -1}, {0, +1, 0}, {0, -1, 0}, /* same level E W S N     */
    {-1, 0, +1}, {+1, 0, +1}, {-1, 0, -1}, {+1, 0, -1}, /* E/W one level up/down */
    {-1, +1, 0}, {+1, +1, 0}, {-1, -1, 0}, {+1, -1, 0}  /* S/N one level up/down */
};

/* the direction of the arc from the neighbour back to v */
static int nb_opposite(int d)
{
    static const int o[14] = {1, 0, 3, 2, 5, 4, 9, 8, 7, 6, 13, 12, 11, 10};
    return o[d];
}

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

/* The skin: every level of the full layout, free or not. */
typedef struct {
    int w, h, m;
    size_t ns, nn;
    const int32_t *lo, *hi;
    uint8_t *free_;         /* level inside its site's window */
    int64_t *ex;            /* balance: excess > 0, deficit < 0 */
    int64_t *res;           /* res[v*14 + d]: residual from v to its free neighbour in d */
    int64_t *ht, *ht2, *ein;
} skin_t;

static size_t sk_node(const skin_t *s, int x, int y, int k)
{
    return (((size_t)k - 1) * s->h + (size_t)y) * s->w + (size_t)x;
}

/* the free neighbour of v in direction d, or -1 */
static int64_t sk_nbr(const skin_t *s, size_t v, int d)
{
    int k = (int)(v / s->ns) + 1;
    int y = (int)((v % s->ns) / s->w), x = (int)(v % s->w);
    int k2 = k + NB[d][0], y2 = y + NB[d][1], x2 = x + NB[d][2];
    if (x2 < 0 || x2 >= s->w || y2 < 0 || y2 >= s->h || k2 < 1 || k2 > s->m - 1) return -1;
    size_t u = sk_node(s, x2, y2, k2);
    return s->free_[u] ? (int64_t)u : -1;
}

static void skin_free(skin_t *s)
{
    free(s->free_); free(s->ex); free(s->res); free(s->ht); free(s->ht2); free(s->ein);
}

/* Folds every arc between a free node and a forced one into the free
 * node's balance: arcs from forced-source levels (and s) are saturated into
 * its excess, arcs into forced-sink levels (and t) become its deficit. */
static int skin_build(skin_t *s, const int32_t *cost, int w, int h, int m, int pen_h, int inh_h,
                      int pen_v, int inh_v, const int32_t *lo, const int32_t *hi)
{
    memset(s, 0, sizeof(*s));
    s->w = w; s->h = h; s->m = m; s->lo = lo; s->hi = hi;
    s->ns = (size_t)w * h;
    s->nn = s->ns * (size_t)(m - 1);
    size_t n1 = s->nn ? s->nn : 1;
    s->free_ = (uint8_t *)calloc(n1, 1);
    s->ex = (int64_t *)calloc(n1, sizeof(int64_t));
    s->res = (int64_t *)calloc(n1 * 14, sizeof(int64_t));
    s->ht = (int64_t *)malloc(n1 * sizeof(int64_t));
    s->ht2 = (int64_t *)malloc(n1 * sizeof(int64_t));
    s->ein = (int64_t *)calloc(n1, sizeof(int64_t));
    if (!s->free_ || !s->ex || !s->res || !s->ht || !s->ht2 || !s->ein) { skin_free(s); return ORC_E_NOMEM; }
    for (int k = 1; k <= m - 1; k++)
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++)
                s->free_[sk_node(s, x, y, k)] = k > lo[y * w + x] && k <= hi[y * w + x];
    for (int k = 1; k <= m - 1; k++)
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                size_t v = sk_node(s, x, y, k);
                if (!s->free_[v]) continue;
                if (k == 1) s->ex[v] += cost[(size_t)y * w + x];                         /* s -> v_1 */
                if (k == m - 1) s->ex[v] -= cost[((size_t)(m - 1) * h + y) * w + x];    /* v_{m-1} -> t */
                for (int d = 0; d < 14; d++) {
                    int k2 = k + NB[d][0], y2 = y + NB[d][1], x2 = x + NB[d][2];
                    if (x2 < 0 || x2 >= w || y2 < 0 || y2 >= h) continue;
                    if (k2 < 1 || k2 > m - 1) continue;        /* the terminals: above */
                    int64_t cout = arc_cap(cost, w, h, x, y, k, d, pen_h, inh_h, pen_v, inh_v);
                    int64_t cin = d == 0 ? ORC_INF
                                : d == 1 ? cost[((size_t)(k - 1) * h + y) * w + x]
                                : arc_cap(cost, w, h, x2, y2, k2, nb_opposite(d), pen_h, inh_h,
                                          pen_v, inh_v);
                    if (k2 <= lo[y2 * w + x2]) s->ex[v] += cin;         /* from a forced-source level */
                    else if (k2 > hi[y2 * w + x2]) s->ex[v] -= cout;    /* into a forced-sink level */
                    else s->res[v * 14 + d] = cout;
                }
            }
    return ORC_OK;
}

/* Exact residual distance of every free node to the nearest node with a
 * deficit (which sit at 1), by breadth-first search backwards over residual
 * arcs; ORC_INF where no deficit is reachable.  `in_block` (optional)
 * restricts the search to arcs between nodes of one block id. */
static int skin_distances(const skin_t *s, int64_t *dist, const int32_t *block_of, int32_t block,
                          const size_t *members, size_t nmem)
{
    size_t count = members ? nmem : s->nn;
    size_t *q = (size_t *)malloc((count ? count : 1) * sizeof(size_t));
    if (!q) return ORC_E_NOMEM;
    size_t qh = 0, qt = 0;
    for (size_t i = 0; i < count; i++) {
        size_t v = members ? members[i] : i;
        dist[v] = ORC_INF;
        if (s->free_[v] && s->ex[v] < 0) { dist[v] = 1; q[qt++] = v; }
    }
    while (qh < qt) {
        size_t v = q[qh++];
        for (int d = 0; d < 14; d++) {
            int64_t u = sk_nbr(s, v, d);
            if (u < 0) continue;
            if (block_of && block_of[u] != block) continue;
            if (dist[u] != ORC_INF) continue;
            /* arc u -> v is the neighbour's arc in the opposite direction */
            if (s->res[(size_t)u * 14 + nb_opposite(d)] > 0) { dist[u] = dist[v] + 1; q[qt++] = (size_t)u; }
        }
    }
    free(q);
    return ORC_OK;
}

/* One synchronous push / relabel step over the given nodes (all free nodes
 * when members is NULL), using the arcs to nodes of the same block only
 * when block_of is given. */
static void skin_step(skin_t *s, int64_t *ht, const int32_t *block_of, int32_t block,
                      const size_t *members, size_t nmem)
{
    size_t count = members ? nmem : s->nn;
    /* push: heights of the step's start, arcs in direction order */
    for (size_t i = 0; i < count; i++) s->ein[members ? members[i] : i] = 0;
    for (size_t i = 0; i < count; i++) {
        size_t v = members ? members[i] : i;
        if (!s->free_[v] || s->ex[v] <= 0 || ht[v] >= ORC_INF) continue;
        int64_t e = s->ex[v];
        for (int d = 0; d < 14 && e > 0; d++) {
            int64_t u = sk_nbr(s, v, d);
            if (u < 0 || (block_of && block_of[u] != block)) continue;
            int64_t r = s->res[v * 14 + d];
            if (r > 0 && ht[u] == ht[v] - 1) {
                int64_t delta = e < r ? e : r;
                s->res[v * 14 + d] -= delta;
                s->res[(size_t)u * 14 + nb_opposite(d)] += delta;
                s->ein[u] += delta;
                e -= delta;
            }
        }
        s->ex[v] = e;
    }
    for (size_t i = 0; i < count; i++) {
        size_t v = members ? members[i] : i;
        s->ex[v] += s->ein[v];
    }
    /* relabel: neighbours' heights of the step's start */
    for (size_t i = 0; i < count; i++) {
        size_t v = members ? members[i] : i;
        s->ht2[v] = ht[v];
        if (!s->free_[v] || s->ex[v] <= 0 || ht[v] >= ORC_INF) continue;
        int64_t hmin = ORC_INF;
        for (int d = 0; d < 14; d++) {
            int64_t u = sk_nbr(s, v, d);
            if (u < 0 || (block_of && block_of[u] != block)) continue;
            if (s->res[v * 14 + d] > 0 && ht[u] < hmin) hmin = ht[u];
        }
        int64_t nh = hmin >= ORC_INF ? ORC_INF : hmin + 1;
        if (nh > ht[v]) s->ht2[v] = nh;
    }
    for (size_t i = 0; i < count; i++) {
        size_t v = members ? members[i] : i;
        ht[v] = s->ht2[v];
    }
}

/* Maximal source side of the current state: labels X_v = lo + number of
 * free levels of the column from which no residual path reaches a node with
 * an unfilled deficit.  Those levels form a prefix of the column. */
static int skin_labels_max_side(const skin_t *s, int32_t *labels)
{
    int rc = skin_distances(s, s->ht2, NULL, 0, NULL, 0);
    if (rc != ORC_OK) return rc;
    for (int y = 0; y < s->h; y++)
        for (int x = 0; x < s->w; x++) {
            int X = s->lo[y * s->w + x], seen_sink = 0;
            for (int k = s->lo[y * s->w + x] + 1; k <= s->hi[y * s->w + x]; k++) {
                int src = s->ht2[sk_node(s, x, y, k)] >= ORC_INF;
                if (src) {
                    if (seen_sink) return ORC_E_PREFIX;
                    X = k;
                } else {
                    seen_sink = 1;
                }
            }
            labels[y * s->w + x] = X;
        }
    return ORC_OK;
}

/* Push-relabel loop of every block on its own (rounds of exact in-block
 * distances and 2n synchronous steps).  Returns ORC_E_TOO_BIG if a block
 * needs more than max_rounds rounds. */
static int skin_blocks(skin_t *s, int b, int max_rounds, int64_t *rounds_out)
{
    int w = s->w, h = s->h, m = s->m;
    int wc = (w + b - 1) / b, hc = (h + b - 1) / b, gc = (m - 1) / b + 1;
    size_t n1 = s->nn ? s->nn : 1;
    int32_t *block_of = (int32_t *)malloc(n1 * sizeof(int32_t));
    int64_t *bh = (int64_t *)malloc(n1 * sizeof(int64_t));
    size_t *mem = (size_t *)malloc((size_t)b * b * b * sizeof(size_t));
    if (!block_of || !bh || !mem) { free(block_of); free(bh); free(mem); return ORC_E_NOMEM; }
    for (size_t v = 0; v < s->nn; v++) {
        int k = (int)(v / s->ns) + 1;
        int y = (int)((v % s->ns) / w), x = (int)(v % w);
        block_of[v] = s->free_[v] ? (int32_t)(((k / b) * hc + y / b) * wc + x / b) : -1;
        bh[v] = ORC_INF;
    }
    int rc = ORC_OK;
    int64_t rounds_total = 0;
    for (int G = 0; G < gc && rc == ORC_OK; G++)
        for (int Y = 0; Y < hc && rc == ORC_OK; Y++)
            for (int X = 0; X < wc && rc == ORC_OK; X++) {
                int32_t id = (G * hc + Y) * wc + X;
                size_t n = 0;
                for (int k = G * b; k < G * b + b && k <= m - 1; k++) {
                    if (k < 1) continue;
                    for (int y = Y * b; y < Y * b + b && y < h; y++)
                        for (int x = X * b; x < X * b + b && x < w; x++) {
                            size_t v = sk_node(s, x, y, k);
                            if (s->free_[v]) mem[n++] = v;
                        }
                }
                if (n == 0) continue;
                int round = 0;
                for (;; round++) {
                    if (round >= max_rounds) { rc = ORC_E_TOO_BIG; break; }
                    if ((rc = skin_distances(s, bh, block_of, id, mem, n)) != ORC_OK) break;
                    int active = 0;
                    for (size_t i = 0; i < n; i++)
                        if (s->ex[mem[i]] > 0 && bh[mem[i]] < ORC_INF) active = 1;
                    if (!active) break;
                    for (size_t t = 0; t < 2 * n; t++) skin_step(s, bh, block_of, id, mem, n);
                }
                rounds_total += round;
            }
    if (rounds_out) *rounds_out = rounds_total;
    free(block_of); free(bh); free(mem);
    return rc;
}

/* Level-2 cut inside given windows: the initialisation, wave_steps synchronous wave
 * steps, then (if blocks) the block-separate push-relabel loops, then the
 * read-out.  excess_out / height_out (optional, full-layout node arrays)
 * receive the state after the wave and before the blocks; rounds_out the
 * total number of block rounds. */
int orc_level2_skin(const int32_t *cost, int w, int h, int m, int pen_h, int inh_h, int pen_v,
                    int inh_v, const int32_t *lo, const int32_t *hi, int b, int wave_steps,
                    int blocks, int32_t *labels, int64_t *excess_out, int64_t *height_out,
                    int64_t *rounds_out)
{
    if (b < 1 || m < 2 || wave_steps < 0 || w < 0 || h < 0) return ORC_E_ARG;
    for (int i = 0; i < w * h; i++)
        if (lo[i] < 0 || hi[i] > m - 1 || lo[i] > hi[i]) return ORC_E_ARG;
    skin_t s;
    int rc = skin_build(&s, cost, w, h, m, pen_h, inh_h, pen_v, inh_v, lo, hi);
    if (rc != ORC_OK) return rc;
    rc = skin_distances(&s, s.ht, NULL, 0, NULL, 0);               /* initialisation */
    for (int t = 1; t <= wave_steps && rc == ORC_OK; t++)            /* wave steps */
        skin_step(&s, s.ht, NULL, 0, NULL, 0);
    if (rc == ORC_OK && excess_out) memcpy(excess_out, s.ex, s.nn * sizeof(int64_t));
    if (rc == ORC_OK && height_out) memcpy(height_out, s.ht, s.nn * sizeof(int64_t));
    if (rounds_out) *rounds_out = 0;
    if (rc == ORC_OK && blocks) rc = skin_blocks(&s, b, 4096, rounds_out);
    if (rc == ORC_OK) rc = skin_labels_max_side(&s, labels);
    skin_free(&s);
    return rc;
}

/* Level-2 approximation: the coarse cut of level 1, its skin windows, then
 * the level-2 cut inside them.  coarse_labels (optional) receives the first
 * cut. */
int orc_approx_level2(const int32_t *cost, int w, int h, int m, int pen_h, int inh_h,
                      int pen_v, int inh_v, int b, int wave_steps, int32_t *labels,
                      int64_t *energy, int32_t *coarse_labels)
{
    if (b < 1 || m < 2) return ORC_E_ARG;
    int wc = (w + b - 1) / b, hc = (h + b - 1) / b, mc = (m + b - 1) / b;
    size_t ns = (size_t)w * h;
    int32_t *cc = (int32_t *)malloc(((size_t)mc * wc * hc + 1) * sizeof(int32_t));
    int32_t *cl = (int32_t *)malloc(((size_t)wc * hc + 1) * sizeof(int32_t));
    int32_t *lo = (int32_t *)malloc((ns + 1) * sizeof(int32_t));
    int32_t *hi = (int32_t *)malloc((ns + 1) * sizeof(int32_t));
    int rc = ORC_E_NOMEM;
    if (cc && cl && lo && hi) {
        int64_t f, e;
        rc = orc_coarse_cost(cost, w, h, m, b, cc);
        if (rc == ORC_OK)
            rc = orc_solve(cc, wc, hc, mc, b * b * pen_h, inh_h, b * b * pen_v, inh_v, 1, cl, &f, &e);
        if (rc == ORC_OK) rc = orc_skin_windows(cl, w, h, m, b, lo, hi);
        if (rc == ORC_OK)
            rc = orc_level2_skin(cost, w, h, m, pen_h, inh_h, pen_v, inh_v, lo, hi, b, wave_steps, 1,
                                 labels, NULL, NULL, NULL);
        if (rc == ORC_OK) *energy = orc_energy(cost, labels, w, h, m, pen_h, inh_h, pen_v, inh_v);
        if (rc == ORC_OK && coarse_labels) memcpy(coarse_labels, cl, (size_t)wc * hc * sizeof(int32_t));
    }
    free(cc); free(cl); free(lo); free(hi);
    return rc;
}

/* Back-most minimiser of E inside per-site windows: the maximal source side
 * of a maximum flow (Dinic) on the windowed graph. */
int orc_solve_window_max_side(const int32_t *cost, int w, int h, int m, int pen_h, int inh_h,
                              int pen_v, int inh_v, const int32_t *lo, const int32_t *hi,
                              int32_t *labels, int64_t *flow)
{
    orc_graph *g = orc_graph_build_window(cost, w, h, m, pen_h, inh_h, pen_v, inh_v, lo, hi);
    if (!g) return ORC_E_NOMEM;
    int rc = orc_maxflow_dinic(g, flow);
    if (rc == ORC_OK) rc = orc_labels_max_side(g, labels);
    orc_graph_free(g);
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

/* ------------------------------------------------------------------------ */
/* Certificate of a solved state in the library's exported layout.           */
/*                                                                          */
/* The state of a full graph (no windows) is given as the balance of every  */
/* node, ex[(k-1)][y][x], and seven stored pair words per node, each an     */
/* int32 [m-1][h][w] array, in this order:                                   */
/*   0 rd   residual of v_k -> v_{k+1} (the data chain; its reverse is      */
/*          unbounded)                                                       */
/*   1 re   residual of v_k -> E_k     (pair total 2 * penalty_h)            */
/*   2 rs   residual of v_k -> S_k     (pair total 2 * penalty_v)            */
/*   3 rem  residual of v_k -> E_{k-1} (pair total inhibit_h; capacity)     */
/*   4 rep  residual of v_k -> E_{k+1} (pair total inhibit_h; capacity 0)   */
/*   5 rsm  residual of v_k -> S_{k-1} (pair total inhibit_v; capacity)     */
/*   6 rsp  residual of v_k -> S_{k+1} (pair total inhibit_v; capacity 0)   */
/* E = (x+1, y), S = (x, y+1).  The terminal arcs are folded into balances  */
/* as in Sec. 4.4: v_1 starts at +g(0), v_{m-1} at -g(m-1).  Everything is    */
/* recomputed here from the definition of the layered graph (Sec. 3,        */
/* Fig. 4); nothing is taken from the solver but the state itself.           */
/* ------------------------------------------------------------------------ */

#define CERT_OK 0
#define CERT_E_BOUNDS 1        /* a residual outside [0, pair total]              */
#define CERT_E_CONSERVATION 2  /* a balance differs from build + net inflow       */
#define CERT_E_NOT_MAXIMUM 3   /* a residual path joins an excess to a deficit    */
#define CERT_E_LABELS 4        /* labels differ from the minimal source side      */
#define CERT_E_VALUE 5         /* flow value differs from E(labels)               */

/* Out-residual of v_k (site x, y) towards its neighbour in direction d (NB
 * order), or -1 when the arc does not exist.  INF for the chain's upward arc. */
static int64_t cert_residual(const int32_t *const *wd, int w, int h, int m, int x, int y, int k,
                             int d, int pen_h, int inh_h, int pen_v, int inh_v)
{
    int k2 = k + NB[d][0], y2 = y + NB[d][1], x2 = x + NB[d][2];
    if (x2 < 0 || x2 >= w || y2 < 0 || y2 >= h || k2 < 1 || k2 > m - 1) return -1;
    size_t here = (((size_t)k - 1) * h + y) * w + x;
    size_t there = (((size_t)k2 - 1) * h + y2) * w + x2;
    switch (d) {
    case 0: return wd[0][here];                        /* down the chain */
    case 1: return ORC_INF;                            /* up the chain */
    case 2: return wd[1][here];                        /* E */
    case 3: return 2 * (int64_t)pen_h - wd[1][there];  /* W: the pair is stored at W */
    case 4: return wd[2][here];                        /* S */
    case 5: return 2 * (int64_t)pen_v - wd[2][there];  /* N */
    case 6: return wd[3][here];                        /* E one level up */
    case 7: return wd[4][here];                        /* E one level down */
    case 8: return (int64_t)inh_h - wd[4][there];      /* W one up: stored at W_{k-1} as its E_{k} */
    case 9: return (int64_t)inh_h - wd[3][there];      /* W one down: stored at W_{k+1} as its E_{k} */
    case 10: return wd[5][here];                       /* S one level up */
    case 11: return wd[6][here];                       /* S one level down */
    case 12: return (int64_t)inh_v - wd[6][there];     /* N one up: stored at N_{k-1} as its S_{k} */
    default: return (int64_t)inh_v - wd[5][there];     /* N one down: stored at N_{k+1} as its S_{k} */
    }
}

/* Checks, in order: (1) every stored word lies in [0, pair total] (the
 * chain word only >= 0: its reverse is unbounded); (2) every balance equals
 * the terminal-arc balance of the build plus the net inflow implied by the
 * words (flow on an arc = capacity - residual); (3) no residual path leads
 * from a node with excess to a node with a deficit (so the preflow is a
 * maximum one); (4) the labels equal the minimal source side (residual
 * reachability from the excess nodes) and (5) the flow value, the sink-arc
 * capacity minus the unfilled deficits, equals E(labels).  flow_out and
 * energy_out receive the recomputed values (when not NULL).  Returns
 * CERT_OK or the number of the first failed check. */
int orc_certify_state(const int32_t *cost, int w, int h, int m, int pen_h, int inh_h, int pen_v,
                      int inh_v, const int32_t *ex, const int32_t *words, const int32_t *labels,
                      int64_t *flow_out, int64_t *energy_out)
{
    if (m < 2 || w < 1 || h < 1) return ORC_E_ARG;
    size_t ns = (size_t)w * h, nn = ns * (size_t)(m - 1);
    const int32_t *wd[7];
    for (int i = 0; i < 7; i++) wd[i] = words + (size_t)i * nn;
    const int64_t total[7] = {-1, 2 * (int64_t)pen_h, 2 * (int64_t)pen_v, inh_h, inh_h, inh_v, inh_v};
    /* (1) bounds; a word of an arc that does not exist is not looked at */
    for (int k = 1; k <= m - 1; k++)
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                size_t v = (((size_t)k - 1) * h + y) * w + x;
                const int exists[7] = {k + 1 <= m - 1, x + 1 < w, y + 1 < h, x + 1 < w && k >= 2,
                                       x + 1 < w && k + 1 <= m - 1, y + 1 < h && k >= 2,
                                       y + 1 < h && k + 1 <= m - 1};
                for (int i = 0; i < 7; i++) {
                    if (!exists[i]) continue;
                    if (wd[i][v] < 0) return CERT_E_BOUNDS;
                    if (total[i] >= 0 && wd[i][v] > total[i]) return CERT_E_BOUNDS;
                }
            }
    /* (2) conservation: balance = build balance + inflow - outflow; each
     * arc pair's flow is counted once, from the end that stores its word */
    int64_t *net = (int64_t *)calloc(nn ? nn : 1, sizeof(int64_t));
    if (!net) return ORC_E_NOMEM;
    int64_t sink_cap = 0;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            net[((size_t)0 * h + y) * w + x] += cost[(size_t)y * w + x];
            int64_t gt = cost[((size_t)(m - 1) * h + y) * w + x];
            net[(((size_t)m - 2) * h + y) * w + x] -= gt;
            sink_cap += gt;
        }
    for (int k = 1; k <= m - 1; k++)
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                size_t v = (((size_t)k - 1) * h + y) * w + x;
                /* stored words: (direction, capacity from v) */
                const int dirs[7] = {0, 2, 4, 6, 7, 10, 11};
                for (int i = 0; i < 7; i++) {
                    int d = dirs[i];
                    int k2 = k + NB[d][0], y2 = y + NB[d][1], x2 = x + NB[d][2];
                    if (x2 < 0 || x2 >= w || y2 < 0 || y2 >= h || k2 < 1 || k2 > m - 1) continue;
                    size_t u = (((size_t)k2 - 1) * h + y2) * w + x2;
                    int64_t cap = d == 0 ? cost[((size_t)k * h + y) * w + x]
                                : d == 2 ? pen_h : d == 4 ? pen_v
                                : d == 6 ? inh_h : d == 10 ? inh_v : 0;
                    int64_t flow = cap - wd[i][v];     /* from v to u (negative: u to v) */
                    net[v] -= flow;
                    net[u] += flow;
                }
            }
    for (size_t v = 0; v < nn; v++)
        if (net[v] != ex[v]) { free(net); return CERT_E_CONSERVATION; }
    free(net);
    /* (3) + (4): residual reachability from the excess nodes */
    uint8_t *mark = (uint8_t *)calloc(nn ? nn : 1, 1);
    size_t *q = (size_t *)malloc((nn ? nn : 1) * sizeof(size_t));
    if (!mark || !q) { free(mark); free(q); return ORC_E_NOMEM; }
    size_t qh = 0, qt = 0;
    for (size_t v = 0; v < nn; v++)
        if (ex[v] > 0) { mark[v] = 1; q[qt++] = v; }
    int rc = CERT_OK;
    while (qh < qt && rc == CERT_OK) {
        size_t v = q[qh++];
        if (ex[v] < 0) { rc = CERT_E_NOT_MAXIMUM; break; }
        int k = (int)(v / ns) + 1, y = (int)((v % ns) / w), x = (int)(v % w);
        for (int d = 0; d < 14; d++) {
            int64_t r = cert_residual(wd, w, h, m, x, y, k, d, pen_h, inh_h, pen_v, inh_v);
            if (r <= 0) continue;
            size_t u = (((size_t)(k + NB[d][0]) - 1) * h + (y + NB[d][1])) * w + (x + NB[d][2]);
            if (!mark[u]) { mark[u] = 1; q[qt++] = u; }
        }
    }
    if (rc == CERT_OK)
        for (int y = 0; y < h && rc == CERT_OK; y++)
            for (int x = 0; x < w; x++) {
                int X = 0;
                while (X < m - 1 && mark[(((size_t)X) * h + y) * w + x]) X++;
                for (int k = X + 2; k <= m - 1; k++)          /* the rest must be off */
                    if (mark[(((size_t)k - 1) * h + y) * w + x]) rc = CERT_E_LABELS;
                if (labels[(size_t)y * w + x] != X) rc = CERT_E_LABELS;
            }
    free(mark); free(q);
    if (rc != CERT_OK) return rc;
    /* (5) max-flow value = min-cut value */
    int64_t unfilled = 0;
    for (size_t v = 0; v < nn; v++) if (ex[v] < 0) unfilled -= ex[v];
    int64_t flow = sink_cap - unfilled;
    int64_t e = orc_energy(cost, labels, w, h, m, pen_h, inh_h, pen_v, inh_v);
    if (flow_out) *flow_out = flow;
    if (energy_out) *energy_out = e;
    return flow == e ? CERT_OK : CERT_E_VALUE;
}

/* The state of the oracle's own graph in the layout above: the residuals of
 * the grid arcs, and as balances the residuals left on the terminal arcs
 * (s -> v_1 positive, v_{m-1} -> t negative) plus the excess a preflow holds
 * at grid nodes (`excess`, indexed by graph node, NULL for a flow), which is
 * the same preflow in the overflow form of Sec. 4.4. */
int orc_graph_export_state(const orc_graph *g, const int64_t *excess, int32_t *ex, int32_t *words)
{
    if (g->lo || g->m < 2) return ORC_E_ARG;
    int w = g->w, h = g->h, m = g->m;
    size_t nn = (size_t)w * h * (size_t)(m - 1);
    memset(ex, 0, nn * sizeof(int32_t));
    memset(words, 0, 7 * nn * sizeof(int32_t));
    const int dirs[7] = {0, 2, 4, 6, 7, 10, 11};
    for (int k = 1; k <= m - 1; k++)
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                size_t v = (((size_t)k - 1) * h + y) * w + x;
                int32_t id = node_id(w, h, x, y, k);
                if (excess) ex[v] += (int32_t)excess[id];
                if (k == 1) {
                    int64_t a = orc_graph_find_arc(g, 0, id);
                    ex[v] += (int32_t)g->res[a];
                }
                if (k == m - 1) {
                    int64_t a = orc_graph_find_arc(g, id, 1);
                    ex[v] -= (int32_t)g->res[a];
                }
                for (int i = 0; i < 7; i++) {
                    int d = dirs[i];
                    int k2 = k + NB[d][0], y2 = y + NB[d][1], x2 = x + NB[d][2];
                    if (x2 < 0 || x2 >= w || y2 < 0 || y2 >= h || k2 < 1 || k2 > m - 1) continue;
                    int64_t a = orc_graph_find_arc(g, id, node_id(w, h, x2, y2, k2));
                    if (a < 0) return ORC_E_ARG;
                    words[(size_t)i * nn + v] = (int32_t)g->res[a];
                }
            }
    return ORC_OK;
}
