/*
 * gazecut.h -- C ABI of the gaze-line stereo graph cut on AMD Instinct MI355X
 * (gfx950).  Method: Oguri & Shibata, "A new stereo formulation not using
 * pixel and disparity models" (arXiv 1803.01516).
 *
 * The library minimises, exactly, the site-labelling energy of Sec. 2
 *
 *     E(X) = sum_v g_v(X_v) + sum_{(u,v) 4-neighbours} h~(X_u - X_v)
 *
 * whose sites are gaze lines (x, y) and whose labels are depth numbers
 * S in [0, m) (Sec. 3; S = 0 is the front), with the convex pairwise term of
 * Sec. 3
 *
 *     h~(d) = penalty * |d| + inhibit * (|d| - 1) * T(|d| > 1).
 *
 * Calls, in pipeline order:
 *   stereo_cost_volume  data term g at every cross point        (Sec. 4.3;
 *                       stereo_cost_volume_rgb: its colour form)
 *   graph_build         layered graph, terminals as overflows    (Sec. 3 Fig. 4, Sec. 4.4)
 *   maxflow_solve       push-relabel with global relabelling     (Sec. 4.4)
 *   extract_labels      minimal source side -> depth numbers, E  (Sec. 3: the cut is the surface)
 *
 * Also: the hierarchical approximations of Sec. 4.5 (coarse_cost_volume,
 * graph_build_skin or graph_build_window, approx_level2_cut), the exact solve
 * warm-started from them (graph_warm_start) and batched solves of many
 * graphs (maxflow_solve_batch, gc_batch_*).
 *
 * Conventions for every call:
 *   - Buffers marked DEVICE are hipMalloc'd (e.g. torch CUDA tensors) and
 *     owned by the caller; the library never allocates or frees device
 *     memory.  Host pointers are read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; results are valid once the stream is
 *     synchronised.  maxflow_solve reads small flags back and so blocks the
 *     calling host thread until the solve has finished.
 *   - Every call returns a gc_status (0 = success, < 0 = error) and never
 *     aborts.  On error no kernel has been enqueued unless the status is
 *     GC_E_HIP or GC_E_NOT_CONVERGED.
 *   - Calls on different graphs may run concurrently on different streams.
 *     Calls that share a graph workspace must be ordered by the caller.
 */
#ifndef GAZECUT_H
#define GAZECUT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GC_OK = 0,
    GC_E_ARG = -1,            /* NULL pointer or invalid option value        */
    GC_E_SHAPE = -2,          /* negative sizes, labels < 1, too many nodes  */
    GC_E_WORKSPACE = -3,      /* workspace smaller than gc_graph_footprint_bytes */
    GC_E_CAP_OVERFLOW = -4,   /* sites*cap + largest pair capacity >= 2^30, or
                                 a data term outside [0, cap] reached the
                                 build: int32 excess/residuals could overflow */
    GC_E_NOT_CONVERGED = -5,  /* iteration cap of gc_solve_opts reached       */
    GC_E_HIP = -6,            /* a HIP runtime call failed (see gc_last_hip_error) */
    GC_E_PREFIX = -7          /* a cut column was not a prefix (internal check) */
} gc_status;

/* Problem description (host struct).  Sites are the width x height gaze
 * lines; labels are the m = `labels` depth numbers.  The cross point of site
 * (x, y) at depth S joins left pixel x - S + (m-1) and right pixel
 * x + S - (m-1) of row y (Sec. 3, Sec. 4.1: one depth step is two pixels of
 * disparity).  `cap` truncates the absolute intensity difference.  The
 * pairwise term uses (penalty_h, inhibit_h) between horizontal neighbours and
 * (penalty_v, inhibit_v) between vertical ones; all four must be >= 0, which
 * is what makes h~ convex (Sec. 2, eq. (1)). */
typedef struct {
    int32_t width;
    int32_t height;
    int32_t labels;
    int32_t cap;
    int32_t penalty_h;
    int32_t inhibit_h;
    int32_t penalty_v;
    int32_t inhibit_v;
} gc_problem;

/* A built graph: a view of the caller's workspace plus the problem. */
typedef struct {
    void *ws;                 /* DEVICE, >= gc_graph_footprint_bytes, 256-B aligned */
    size_t ws_bytes;
    gc_problem p;
    int32_t window_block;     /* 0: full graph; b > 0: thin-skin graph of block size b */
    int32_t compact;          /* thin skin storing only each site's window of levels
                                 (graph_build_skin); 0 otherwise */
} gc_graph;

/* Solver options; a zero-filled struct selects the defaults. */
typedef struct {
    int32_t relabel_period;   /* most push-relabel sweeps between global relabels (default 24
                                 when the full problem has fewer than 32 levels, else 32) */
    int32_t max_sweeps;       /* give up with GC_E_NOT_CONVERGED after this many (default 1<<20) */
    int32_t tile_w;           /* BFS tile extent along x (default 8)           */
    int32_t tile_h;           /* along y (default 8)                          */
    int32_t tile_j;           /* along the depth-number axis (default 16)     */
    int32_t local_iters;      /* max in-tile relaxation rounds per pass (default 4 below 32
                                 stored levels, else 8; 8 in a compact thin skin) */
    int32_t flags;            /* GC_OPT_* bits                                */
    int32_t relabel_passes;   /* most relaxation passes of a global relabel that
                                 does not end the solve (default 8 when the full
                                 problem has fewer than 32 levels, 16 from there
                                 on, a thin skin following its full problem;
                                 < 0: none stops early;
                                 only a solve's first 24 relabels may).  Stopped early, its heights bound the
                                 distances from above near the deficits and are
                                 INF farther away (those nodes wait for the next
                                 relabel); a relabel that then finds no active
                                 node is carried on to its exact fixpoint, so the
                                 solve still ends on an exact one. */
} gc_solve_opts;

/* gc_solve_opts.flags: bracket one launch in 16 (one in 4 on graphs of 4 M
 * nodes or more) of each kernel class (chosen by a hash
 * of its number, so the sample does not alias with the sweep periods) with a
 * pair of hipEvents on the solve stream; gc_solve_stats then holds every
 * class's launch count and its device time estimated as the mean of the timed
 * launches times that count (timing every launch would slow the host enough
 * to leave the GPU idle between short sweeps). */
#define GC_OPT_TIME_KERNELS 1

/* gc_solve_opts.flags: replay the push-relabel sweeps of a relabel period
 * from a captured hipGraph (needs a non-null stream; ignored with
 * GC_OPT_TIME_KERNELS).  maxflow_solve keeps the last few captures per host
 * thread, keyed by the graph's workspace, shape and the sweep options. */
#define GC_OPT_SWEEP_GRAPH 2

/* gc_solve_opts.flags: run the wave-front pass of Sec. 4.4 once before the
 * first global relabel (each column hands its excess along the data chain
 * towards the sink as far as the chain's residuals allow, in one pass per
 * column).  Off by default.  Labels, energy and flow do not depend on it. */
#define GC_OPT_WAVE_FIRST 4

/* gc_solve_opts.flags: the sweep kernels.  FUSED_SWEEP (the default) runs
 * one fused push-relabel kernel per sweep, SPLIT_SWEEP a push kernel and a
 * relabel kernel (it wins when both are given).  The final result does not
 * depend on it. */
#define GC_OPT_FUSED_SWEEP 16
#define GC_OPT_SPLIT_SWEEP 64

/* gc_solve_opts.flags, maxflow_solve: by default the first period runs
 * relabel_period sweeps and each later one twice the largest height of an
 * active node at the global relabel before it (at least 16, at most
 * relabel_period); FIXED_PERIOD runs relabel_period sweeps every time.
 * Batched merged rounds always run full periods. */
#define GC_OPT_FIXED_PERIOD 32

/* gc_solve_opts.flags: work-list launches for single graphs.  Every sweep
 * runs over the 256-node blocks a compaction launch lists as holding an
 * active node (or inflow), and every relaxation pass over the tiles whose
 * neighbourhood changed in the pass before, each on a fixed grid of
 * workgroups.  Off by default (one workgroup per block or tile of the whole
 * graph): measured slower on single graphs.  The result does not depend on
 * it. */
#define GC_OPT_LISTS 256

/* Kernel classes of gc_solve_stats.kernel_ms / kernel_launches. */
#define GC_K_PUSH 0           /* push sweep, or fused push-relabel sweep       */
#define GC_K_RELABEL 1        /* relabel sweep (also merges inflow)           */
#define GC_K_RELAX 2          /* one tiled BFS relaxation pass                */
#define GC_K_OTHER 3          /* arc masks, BFS seeds, active count           */
#define GC_K_CLASSES 4

/* Solver statistics (host struct, filled by maxflow_solve). */
typedef struct {
    int64_t pushes;           /* arc pushes that moved a positive amount      */
    int32_t sweeps;           /* push + relabel sweeps over the graph         */
    int32_t global_relabels;  /* exact distance recomputations                */
    int32_t bfs_passes;       /* tiled relaxation passes (all BFS work)       */
    int32_t active_last;      /* active nodes at the last check (0 when done) */
    int32_t kernel_launches[GC_K_CLASSES];  /* with GC_OPT_TIME_KERNELS only */
    double kernel_ms[GC_K_CLASSES];         /* estimated device time per class */
    double done_ms;           /* maxflow_solve_batch: host ms from its start to this graph's end */
    int64_t active_visits;    /* nodes with excess and a finite height met by the
                                 push (split) or fused sweeps, summed over sweeps */
} gc_solve_stats;

/* Largest number of graphs one batch holds at a time. */
#define GC_BATCH_MAX_GRAPHS 256

/* Human-readable name of a status code (static string). */
const char *gc_status_str(int status);

/* Last HIP error code seen by the calling thread (0 if none). */
int gc_last_hip_error(void);

/* Validates a problem: GC_OK, GC_E_ARG, GC_E_SHAPE or GC_E_CAP_OVERFLOW. */
int gc_problem_check(const gc_problem *p);

/* Bytes of DEVICE workspace graph_build needs for `p` (0 if p is invalid).
 * Linear in the number of graph nodes width*height*(labels-1); used both to
 * allocate and to admit work by its memory footprint. */
size_t gc_graph_footprint_bytes(const gc_problem *p);

/* Data term of Sec. 4.3 for grayscale pairs:
 *   cost[(S*height + y)*width + x] = min(|left(y, x-S+m-1) - right(y, x+S-m+1)|, cap)
 * and cap when either pixel falls outside the image.
 * left, right: DEVICE uint8 [height][width], row-major, rectified pair.
 * cost:        DEVICE int32 [labels][height][width] (label-major), written.
 * Errors: GC_E_ARG (NULL), GC_E_SHAPE, GC_E_HIP. */
int stereo_cost_volume(const uint8_t *left, const uint8_t *right, const gc_problem *p,
                       int32_t *cost, void *stream);

/* The colour data term of Sec. 4.3: g(x, y, S) = min(|dR| + |dG| + |dB|,
 * p->cap) over the two pixels of the cross point (0..765; cap >= 765 leaves
 * it untruncated, the paper's form, used with penalty 14 and inhibit 1023),
 * cap outside the image.
 * left, right: DEVICE uint8 [height][width][3], channels interleaved.
 * cost:        DEVICE int32 [labels][height][width] (label-major), written.
 * Errors: GC_E_ARG (NULL), GC_E_SHAPE, GC_E_HIP. */
int stereo_cost_volume_rgb(const uint8_t *left, const uint8_t *right, const gc_problem *p,
                           int32_t *cost, void *stream);

/* Builds the layered graph of Sec. 3 (Fig. 4) in `ws`: for every site the
 * nodes v_1..v_{m-1} ("v_k on the source side" means X_v >= k) with the data
 * chain v_k -> v_{k+1} of capacity g(k) and an unbounded reverse arc,
 * same-level arcs of capacity penalty both ways and the diagonal arcs
 * u_{k+1} -> v_k of capacity inhibit between 4-neighbours.  The terminal
 * arcs are folded into node overflows as in Sec. 4.4: v_1 starts with excess
 * g(0) and v_{m-1} with deficit g(m-1).
 * cost: DEVICE int32 [labels][height][width] from stereo_cost_volume, or any
 *       data term of the same layout whose values lie in [0, p->cap]; read
 *       only.  The int32 bounds on flow and excess rest on that range: the
 *       build flags a value outside it on the device, and maxflow_solve,
 *       extract_labels and approx_level2_cut on the graph then return
 *       GC_E_CAP_OVERFLOW (graph_build itself does not wait for the device).
 * ws:   DEVICE workspace of at least gc_graph_footprint_bytes(p) bytes,
 *       256-byte aligned; fully (re)initialised, so a graph can be rebuilt
 *       in place.
 * g_out: host struct filled with (ws, ws_bytes, *p).
 * Errors: GC_E_ARG, GC_E_SHAPE, GC_E_CAP_OVERFLOW, GC_E_WORKSPACE, GC_E_HIP. */
int graph_build(const gc_problem *p, const int32_t *cost, void *ws, size_t ws_bytes,
                gc_graph *g_out, void *stream);

/* Exact maximum preflow by parallel push-relabel with global relabelling
 * (Sec. 4.4): alternating push and relabel sweeps over all nodes, with an
 * exact residual-distance recomputation every `relabel_period` sweeps; stops
 * when no node with excess can reach a node with deficit.  The state left in
 * the workspace is what extract_labels reads.
 * o: host options or NULL for defaults; stats: host struct or NULL.
 * Errors: GC_E_ARG, GC_E_NOT_CONVERGED (state is a valid preflow but not a
 * maximum one), GC_E_CAP_OVERFLOW (the graph was built from a data term
 * outside [0, cap]; found at the first global relabel), GC_E_HIP. */
int maxflow_solve(gc_graph *g, const gc_solve_opts *o, gc_solve_stats *stats, void *stream);

/* Reads the minimum cut off a solved graph.  The source side is every node
 * reachable by residual arcs from a node that still has excess; this is the
 * minimal source side of all minimum cuts, so the labelling is the unique
 * front-most optimal surface (Sec. 3: the cut is the surface of real cross
 * points).  X_v = number of source-side nodes in the column of v.
 * cost:   DEVICE int32 [labels][height][width], the same data term the graph
 *         was built from (used to evaluate E).
 * labels: DEVICE int32 [height][width], written.
 * result: DEVICE int64[2], written: result[0] = E(labels) evaluated from its
 *         definition, result[1] = value of the maximum flow.  The two are
 *         equal when the solve finished (max-flow = min-cut).
 * Errors: GC_E_ARG, GC_E_PREFIX, GC_E_CAP_OVERFLOW (data term outside
 * [0, cap] at the build), GC_E_HIP. */
int extract_labels(const gc_graph *g, const int32_t *cost, int32_t *labels,
                   int64_t *result, void *stream);

/* Copies a graph's state out in a documented layout, for checking it
 * independently of the library (e.g. the certificate of a maximum preflow:
 * capacity bounds, conservation against the build, no residual path from an
 * excess to a deficit).  excess: DEVICE int32 [labels-1][height][width], the
 * node balances with the terminal arcs folded in as in Sec. 4.4 (v_1 starts
 * at +g(0), v_{m-1} at -g(m-1)).  words: DEVICE int32
 * [7][labels-1][height][width], the stored residual of one arc of each arc
 * pair, in this order (E = x+1, S = y+1; pair totals in brackets):
 *   0 v_k -> v_{k+1}  (reverse unbounded)   1 v_k -> E_k   (2 penalty_h)
 *   2 v_k -> S_k      (2 penalty_v)         3 v_k -> E_{k-1} (inhibit_h)
 *   4 v_k -> E_{k+1}  (inhibit_h)           5 v_k -> S_{k-1} (inhibit_v)
 *   6 v_k -> S_{k+1}  (inhibit_v)
 * Words of arcs that do not exist (image border, k out of range) are 0.  For
 * a thin-skin graph the levels outside the windows are inert and their
 * entries carry no meaning.  Errors: GC_E_ARG, GC_E_HIP. */
int gc_graph_state(const gc_graph *g, int32_t *excess, int32_t *words, void *stream);

/* ------------------------------------------------------------------------
 * Hierarchical approximation, level 1 (Sec. 4.5).  b x b x b neighbouring
 * cross points form one delegate point; a first exact cut on the delegate
 * points decides which of them hold the surface, and a second exact cut
 * finds the real cross points inside the thin skin around it.  Pipeline:
 *   gc_coarse_problem -> coarse_cost_volume -> graph_build -> maxflow_solve
 *   -> extract_labels (delegate labels) -> graph_build_window ->
 *   maxflow_solve -> extract_labels (fine labels, exact E of the result).
 * Block size 1 reproduces the exact minimisation.
 * ---------------------------------------------------------------------- */

/* Delegate-point problem of block size `block` (host only): ceil(w/b) x
 * ceil(h/b) sites and ceil(m/b) labels; coarse site (X, Y) covers sites
 * x / b = X, y / b = Y, coarse label Sc covers S / b = Sc.  cap and penalties
 * scale by b*b (a one-group step between coarse sites stands for a ramp of b
 * depth numbers over b rows of fine pairs); inhibit is unchanged.
 * Errors: GC_E_ARG (block < 1), the errors of gc_problem_check. */
int gc_coarse_problem(const gc_problem *p, int32_t block, gc_problem *coarse);

/* Delegate-point data term: coarse_cost[(Sc*hc + Y)*wc + X] = sum over the
 * sites of coarse site (X, Y) of min over S in group Sc of cost(x, y, S).
 * cost: DEVICE int32 [labels][height][width]; coarse_cost: DEVICE int32
 * [ceil(m/b)][ceil(h/b)][ceil(w/b)], written. */
int coarse_cost_volume(const gc_problem *p, const int32_t *cost, int32_t block,
                       int32_t *coarse_cost, void *stream);

/* Thin-skin graph (Sec. 4.5, second cut): like graph_build on the full
 * problem, but site (x, y) may only take labels in
 *   [max(0, b*(Sc-1)), min(m-1, b*(Sc+2)-1)],  Sc = coarse_labels[y/b][x/b],
 * the delegate group of the first cut and the groups directly above and
 * below.  Levels outside the window are forced to the source (above) or sink
 * (below) side and their arcs are folded into overflows.  maxflow_solve and
 * extract_labels accept the result; extract_labels then returns the exact
 * energy of the restricted optimum, and result[1] the restricted min-cut
 * value (equal to it).
 * coarse_labels: DEVICE int32 [ceil(h/b)][ceil(w/b)] labels in [0, ceil(m/b)).
 * ws: as for graph_build (same footprint). */
int graph_build_window(const gc_problem *p, const int32_t *cost, const int32_t *coarse_labels,
                       int32_t block, void *ws, size_t ws_bytes, gc_graph *g_out, void *stream);

/* The same thin skin, stored compactly: only the window's levels of each
 * site, min(3b - 1, m - 1) per site (level t of site (x, y) is level
 * wlo + t of the full graph, wlo the bottom of its window above; stored
 * levels beyond a clamped window are inert padding), so the second cut's
 * sweeps, masks and relaxation passes cover the free nodes only.  The arcs
 * between forced nodes, which every labelling cuts, are summed at the build.
 * maxflow_solve, extract_labels, approx_level2_cut and graph_warm_start
 * (as `skin`) accept it, with the same results as for graph_build_window;
 * gc_graph_state and the batch (gc_batch_add, maxflow_solve_batch with
 * GC_OPT_BATCH_MERGED) do not (GC_E_ARG).
 * ws: >= gc_skin_footprint_bytes(p, block), 256-B aligned.
 * Errors: as graph_build_window; GC_E_ARG also when min(3b - 1, m - 1) > 16. */
int graph_build_skin(const gc_problem *p, const int32_t *cost, const int32_t *coarse_labels,
                     int32_t block, void *ws, size_t ws_bytes, gc_graph *g_out, void *stream);

/* Bytes of DEVICE workspace graph_build_skin needs (0 for block < 1 or an
 * invalid problem). */
size_t gc_skin_footprint_bytes(const gc_problem *p, int32_t block);

/* Coarse-to-fine warm start of the exact solve (our design next to the
 * hierarchy of Sec. 4.5): seeds a freshly built full graph `g` with the
 * state of a thin-skin graph `skin` of the same problem and data term that
 * maxflow_solve has solved.  Free skin nodes keep their excess and the pair
 * words of their arcs; the arcs the skin folded into overflows (from
 * forced-source levels into the skin, from the skin into forced-sink levels)
 * carry their capacity in the full graph, so forced-source nodes start with
 * the deficit and forced-sink nodes with the excess of what they exchanged;
 * every other arc keeps the build's value.  The result is a pseudoflow
 * (capacities respected, nodes may hold a deficit anywhere), which the
 * solver handles as it handles the sink deficits: maxflow_solve on `g` then
 * ends in the same maximum flow value and extract_labels in the same minimal
 * minimum cut as from the cold build (the minimal source side is unique).
 * g:    built by graph_build (not a skin) on the same gc_problem;
 * skin: built by graph_build_window or graph_build_skin and solved; read only;
 * cost: DEVICE int32 [labels][height][width], the data term of both.
 * Waits for the device (one 8-byte read-back).
 * Errors: GC_E_ARG (wrong graph kinds or problems), GC_E_CAP_OVERFLOW (the
 * seeded excess totals 2^30 or more, beyond the int32 bound of one node's
 * excess), GC_E_HIP. */
int graph_warm_start(gc_graph *g, const gc_graph *skin, const int32_t *cost, void *stream);

/* Level-2 approximation (Sec. 4.5) on a thin-skin graph from
 * graph_build_window or graph_build_skin (block size b = skin->window_block,
 * 1 <= b <= 4): the
 * wave-front pre-phase covers the whole skin and the push-relabel loop cuts
 * every block separately.  Readings (the paper omits the details):
 *   - the wave front is an initialisation (exact residual distances to the
 *     deficits) and `wave_steps` synchronous steps over the skin: every node
 *     with excess and a finite height pushes, arc by arc in a fixed order,
 *     to neighbours exactly one below, then every node holding excess is
 *     lifted to one above its lowest residual neighbour (heights of the
 *     step's start: the result does not depend on the schedule);
 *   - a block is the b x b x b cross points of one delegate point: the free
 *     levels k with k / b equal to one label group, over the b x b sites of
 *     the delegate point; its push-relabel loop uses only the arcs between
 *     its own nodes and runs rounds (exact in-block distances, then 2n
 *     synchronous steps of the same rule, n its nodes) until no node with
 *     excess reaches an in-block deficit;
 *   - the cut is read as the maximal source side of the final state: a
 *     level is on the sink side iff a residual path leads from it to an
 *     unfilled deficit.
 * With a wave long enough to reach a maximum preflow the result is the
 * back-most minimum of E inside the windows.
 * cost:          DEVICE int32 [labels][height][width], the full data term.
 * coarse_labels: DEVICE int32 [ceil(h/b)][ceil(w/b)], the delegate labels
 *                the skin was built from.
 * wave_steps:    A-1 >= 0; max(32, labels) recommended (fewer steps can leave
 *                regions whose flow has not reached the cut at the top of
 *                their windows).
 * labels:        DEVICE int32 [height][width], written.
 * result:        DEVICE int64[2], written: result[0] = E(labels) from its
 *                definition, result[1] = -1 (no global cut value exists).
 * The skin's state is consumed.  Errors: GC_E_ARG (not a thin-skin graph,
 * b^3 > 64, wave_steps < 0), GC_E_NOT_CONVERGED (a block needed more than
 * 4096 rounds), GC_E_PREFIX, GC_E_CAP_OVERFLOW (data term outside [0, cap]
 * at the build), GC_E_HIP. */
int approx_level2_cut(gc_graph *skin, const int32_t *cost, const int32_t *coarse_labels,
                      int32_t wave_steps, int32_t *labels, int64_t *result, void *stream);

/* ------------------------------------------------------------------------
 * Batched solve.  Many graphs of any sizes (full or thin-skin) are solved
 * together, each advancing through the single-graph sequence (exact global
 * relabel by relaxation passes, termination test, a period of push-relabel
 * sweeps) on the device.  A step moves every member by one phase of that
 * sequence in four launches shared by all members: one workgroup per member
 * picks its next phase from what its last step left, the members' work lists
 * are compacted (active blocks of a sweep, changed tiles of a relaxation
 * pass), their offsets are summed, and a fixed grid of workgroups takes the
 * units of all members in turn (the work queue).  A round replays a captured
 * run of steps and reads the members' records once.  Results are identical
 * to maxflow_solve on each graph (the cut is canonical).  Graphs may join
 * between rounds, which is how a serving loop admits new work while others
 * are on the GPU.
 * ---------------------------------------------------------------------- */

/* Opaque host object of a batch (allocated by gc_batch_create). */
typedef struct gc_batch gc_batch;

/* Bytes of DEVICE memory a batch needs for its graph table (256-B aligned). */
size_t gc_batch_footprint_bytes(void);

/* Creates a batch over the caller's DEVICE table buffer; `o` fixes the
 * relabel period, relaxation tile (8x8x16, 16x8x16, 8x8x32 or 16x16x8),
 * sweep kind and max_sweeps for all members; GC_OPT_WAVE_FIRST is not used.
 * Errors: GC_E_ARG (also for another tile shape), GC_E_WORKSPACE. */
int gc_batch_create(void *dev_table, size_t dev_bytes, const gc_solve_opts *o, gc_batch **out);

/* Frees the host object (not the caller's memory). */
int gc_batch_destroy(gc_batch *b);

/* Number of graphs currently in the batch. */
int gc_batch_members(const gc_batch *b);

/* Adds a built graph (graph_build or graph_build_window), identified by
 * `tag`.  Its workspace must stay untouched until it leaves the batch.
 * Errors: GC_E_ARG (batch full), errors of an invalid graph. */
int gc_batch_add(gc_batch *b, const gc_graph *g, int64_t tag);

/* One round on `stream`: 32 steps of every member (captured once per
 * membership and replayed when `stream` is not null), then one read-back of
 * the members' records.  Members that finished leave the batch; their tags
 * (and stats, if done_stats is not NULL) are written to done_tags[0 ..
 * *n_done-1] (at most max_done of them; others are reported by the next
 * call).  A member stops unfinished after max_sweeps sweeps, with
 * stats.active_last > 0.  Returns with the stream synchronised.
 * Errors: GC_E_ARG, GC_E_HIP. */
int gc_batch_round(gc_batch *b, void *stream, int64_t *done_tags, gc_solve_stats *done_stats,
                   int32_t max_done, int32_t *n_done);

/* Concurrent lanes of maxflow_solve_batch (host threads, one HIP stream each). */
#define GC_BATCH_LANES 4

/* Batch engines of maxflow_solve_batch with GC_OPT_BATCH_MERGED. */
#define GC_BATCH_ENGINES 3

/* gc_solve_opts.flags, maxflow_solve_batch: run the graphs in rounds of the
 * batch engine (gc_batch_*: every member advances on the device, each step's
 * launches shared by all members; on `stream`, using dev_table) instead of
 * concurrent lanes. */
#define GC_OPT_BATCH_MERGED 128

/* Solves n built graphs and returns when all are solved; extract_labels then
 * reads each.  By default the graphs go, largest first, to GC_BATCH_LANES
 * concurrent lanes: host threads that each own a HIP stream (default
 * priority) and solve one graph at a time exactly as maxflow_solve does, so
 * one graph's latency-bound phases (relaxation passes, read-backs) overlap
 * other graphs' sweeps; dev_table may then be NULL.  With
 * GC_OPT_BATCH_MERGED the graphs, largest first, are dealt to up to
 * GC_BATCH_ENGINES batch engines (gc_batch_*), the first on `stream`, the
 * others on streams of their own, all driven from the calling thread (every
 * engine's round is queued before any is waited for) and refilled as members
 * finish; dev_table holds one table of gc_batch_footprint_bytes() per engine
 * (dev_bytes decides how many run, at least one).
 * Either way the work starts after what is queued on `stream` so far.  stats
 * (optional) receives n entries in input order.  Returns GC_E_NOT_CONVERGED
 * if any graph hit max_sweeps, else the first error of any graph. */
int maxflow_solve_batch(gc_graph *const *gs, int32_t n, void *dev_table, size_t dev_bytes,
                        const gc_solve_opts *o, gc_solve_stats *stats, void *stream);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc: work recorded under stream capture, tight serving loops,
 * harnesses that forbid allocation).
 *
 * gc_solve_pair_static runs the exact path of one pair, the sequence
 * stereo_cost_volume -> graph_build -> maxflow_solve -> extract_labels, with
 * the cost volume and the graph's workspace in a static device array of
 * GC_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (looked up once per device on the first call there).
 * It calls no hipMalloc, hipFree, hipHostMalloc or other allocating routine;
 * read-backs land in pageable host memory on the caller's stack.
 * left, right: DEVICE uint8 [height][width] as for stereo_cost_volume.
 * o:      host options or NULL; GC_OPT_TIME_KERNELS and GC_OPT_SWEEP_GRAPH
 *         are refused (GC_E_ARG): they create events or graphs.
 * labels: DEVICE int32 [height][width], written.
 * result: DEVICE int64[2], written as by extract_labels.
 * stats:  host struct or NULL, as for maxflow_solve.
 * The device whose array is used is the current one; stream must belong to
 * it.  Every call on one GPU shares that GPU's array, and the array keeps the
 * last call's contents (the path initialises every byte it reads): calls that
 * overlap on one GPU, on any streams or host threads, race and must be
 * serialised by the caller.
 * Errors: GC_E_WORKSPACE when gc_solve_pair_static_bytes(p) exceeds
 * GC_STATIC_SCRATCH_BYTES, the errors of the four calls it stands for,
 * GC_E_HIP when the array's device address cannot be found. */
#define GC_STATIC_SCRATCH_BYTES (96u << 20)

/* Bytes of the static array one pair of `p` needs (cost volume + graph
 * workspace, 256-byte aligned); 0 for an invalid problem.  About 83 MB at
 * 384x288x16. */
size_t gc_solve_pair_static_bytes(const gc_problem *p);

int gc_solve_pair_static(const uint8_t *left, const uint8_t *right, const gc_problem *p,
                         const gc_solve_opts *o, int32_t *labels, int64_t *result,
                         gc_solve_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GAZECUT_H */
