// gazecut.hip -- HIP kernels and C ABI for the gaze-line stereo graph cut
// (Oguri & Shibata, arXiv 1803.01516) on MI355X / gfx950.
//
// Graph state lives in one caller-owned workspace as label-major
// structure-of-arrays int32 words, node index n = (j*H + y)*W + x with
// j = k-1 the depth layer (k = 1..m-1), so consecutive threads touch
// consecutive x and every access of a sweep is coalesced.  Per node:
//
//   ex   excess (terminal arcs folded into overflows, Sec. 4.4)
//   ht   height (distance label of push-relabel)
//   rd   residual of v_k -> v_{k+1}         (data chain; reverse is unbounded)
//   re   residual of v_k -> E_k             pair total 2*penalty_h
//   rs   residual of v_k -> S_k             pair total 2*penalty_v
//   rem  residual of v_k -> E_{k-1}         pair total inhibit_h
//   rep  residual of v_k -> E_{k+1}         pair total inhibit_h
//   rsm  residual of v_k -> S_{k-1}         pair total inhibit_v
//   rsp  residual of v_k -> S_{k+1}         pair total inhibit_v
//
// Each arc pair is stored once; the opposite residual is the pair total
// minus the stored word.  E/S are the (x+1, y) and (x, y+1) neighbours.
//
// Push-relabel runs as synchronous sweeps.  In the push sweep heights are
// read-only, so along any arc pair at most one endpoint is admissible
// (h(u) = h(v) + 1 excludes h(v) = h(u) + 1): each pair word has a single
// writer and needs no atomic.  Inflow goes to a separate `ein` array with
// atomics and is merged by the relabel sweep.  Relabels only raise heights,
// so the concurrent reads of neighbour heights in the relabel sweep see
// lower bounds and the labelling stays valid.
//
// Global relabelling and the cut read-out are both min-plus fixpoints over
// a 14-bit residual arc mask per node: BFS distance to the deficit nodes
// (step 1) and reachability from the excess nodes (step 0).  They run as
// LDS-tiled relaxations: each workgroup iterates its site x layer tile to a
// local fixpoint, and passes repeat until no tile changes.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <type_traits>
#include <vector>

#include "gazecut.h"

#define GC_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int32_t kInf = 1 << 30;
constexpr int kBlock = 256;
constexpr int kSkinMaxLevels = 16;      // levels per site of a compact thin skin (3b - 1, b <= 5)
constexpr int kMaxFlags = 16;

// Arc directions (bit index in the residual masks) and their offsets
// (dj, dy, dx).  opposite(d) = d ^ 1 for 0..5; 6<->9, 7<->8, 10<->13, 11<->12.
enum Dir {
    D_DOWN = 0, D_UP = 1, D_E = 2, D_W = 3, D_S = 4, D_N = 5,
    D_EM = 6, D_EP = 7, D_WM = 8, D_WP = 9, D_SM = 10, D_SP = 11, D_NM = 12, D_NP = 13
};
__host__ __device__ constexpr int dir_dj(int d)
{
    return d == D_DOWN ? 1 : d == D_UP ? -1
         : (d == D_EM || d == D_WM || d == D_SM || d == D_NM) ? -1
         : (d == D_EP || d == D_WP || d == D_SP || d == D_NP) ? 1 : 0;
}
__host__ __device__ constexpr int dir_dy(int d)
{
    return (d == D_S || d == D_SM || d == D_SP) ? 1 : (d == D_N || d == D_NM || d == D_NP) ? -1 : 0;
}
__host__ __device__ constexpr int dir_dx(int d)
{
    return (d == D_E || d == D_EM || d == D_EP) ? 1 : (d == D_W || d == D_WM || d == D_WP) ? -1 : 0;
}

// Bits of DevHeader::prefix_err: 1 a column's source side is not a prefix,
// 2 a level-2 block loop hit its round cap, kCostErr a data term outside
// [0, cap] reached graph_build.
constexpr int32_t kCostErr = 4;

struct DevHeader {
    int32_t flags[kMaxFlags];
    int32_t active;
    int32_t prefix_err;
    int32_t max_height;       // largest height of an active node at the last count
    int32_t lists[4];         // lengths of the block list (0, 1) and the tile list (2, 3)
    int32_t pad[9];
    unsigned long long pushes;
    unsigned long long visits;  // active nodes visited by the push (or fused) sweeps
    long long tcap;           // capacity of all arcs into the sink side
    long long c0;             // capacity of arcs from forced-source to forced-sink nodes
    long long seeded;         // total positive excess of a warm-started state
    unsigned long long pad2[11];
};
static_assert(sizeof(DevHeader) == 256, "header must stay 256 bytes");

// Reduction targets, one 64-byte line each: a block adds its partial sum to
// slot blockIdx % kSlots, so no single address takes every block's atomic.
struct Slot {
    unsigned long long pushes;
    long long e0, e1;
    int32_t active;
    int32_t max_height;
    long long tcap, c0;
    unsigned long long visits;
    long long pad2[1];
};
static_assert(sizeof(Slot) == 64, "one slot per cache line");
constexpr int kSlots = 256;

// Device memory of a graph.  The pointers carry the global address space, so
// kernels that read a graph from a table (the batch engine) access its arrays
// with global instructions, as kernels whose graph is an argument do; a
// pointer of unknown space compiles to flat instructions, whose waits also
// wait for scalar loads.
// (The host pass sees plain pointers of the same size and value.)
#if defined(__HIP_DEVICE_COMPILE__)
#define GDEV __attribute__((address_space(1)))
#else
#define GDEV
#endif

struct Graph {
    GDEV int32_t *ex, *ht, *rd, *re, *rs, *rem, *rep, *rsm, *rsp, *ein, *aux;
    GDEV uint16_t *mask;
    GDEV int32_t *stamps;     // per relaxation tile: last pass that changed it
    GDEV int32_t *blist, *tlist;   // work lists: 256-node blocks of a sweep, tiles of a relaxation pass
    GDEV int32_t *wlo, *whi;  // per-site label window of a thin-skin graph
    GDEV uint8_t *bact;       // per 64-node group: holds an active node
    GDEV uint8_t *binf;       // per 64-node group: received inflow in the last push sweep
    GDEV DevHeader *hdr;
    GDEV Slot *slots;
    int32_t W, H, J;
    int64_t plane, N;
    int32_t te, ts, ie, is;   // pair totals: 2*pen_h, 2*pen_v, inh_h, inh_v
    int32_t win;              // thin-skin graph (levels outside per-site windows are inert)
    int32_t cw;               // compact thin skin: level t of site (x, y) is level wlo + t, and
                              // only the window's levels are stored (J of them per site)
    int32_t Jf;               // levels of the full graph (m - 1)
};

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Levels stored per site: m - 1 for a full graph (or a thin skin in the full
// layout), the window's 3b - 1 (at most m - 1) for a compact thin skin of
// block size b.
int64_t stored_levels(const gc_problem *p, int compact_block)
{
    const int64_t J = p->labels > 0 ? p->labels - 1 : 0;
    return compact_block > 0 ? std::min<int64_t>(J, 3 * (int64_t)compact_block - 1) : J;
}

// Activity flags cover 64-node groups, the nodes of one wavefront of a
// block, so that each wavefront decides, clears and sets its own flags with
// no barrier.  Every block has four, also past the last node.
constexpr int kGroup = 64;
inline size_t flag_bytes(int64_t n) { return (size_t)((n + kBlock - 1) / kBlock) * (kBlock / kGroup); }

thread_local int t_last_hip = 0;

bool hip_ok(hipError_t e)
{
    if (e != hipSuccess) { t_last_hip = (int)e; return false; }
    return true;
}

int64_t node_count(const gc_problem *p, int compact_block = 0)
{
    return (int64_t)p->width * p->height * stored_levels(p, compact_block);
}

// Relaxation tiles are at least 8 x 4 x 4 nodes, which bounds the tile count.
constexpr int kMinTileW = 8, kMinTileH = 4, kMinTileJ = 4;
size_t max_tiles(const gc_problem *p, int compact_block = 0)
{
    const int64_t J = stored_levels(p, compact_block);
    return (size_t)(((int64_t)p->width + kMinTileW - 1) / kMinTileW) *
           (size_t)(((int64_t)p->height + kMinTileH - 1) / kMinTileH) *
           (size_t)((J + kMinTileJ - 1) / kMinTileJ);
}

Graph view(const gc_graph *g)
{
    const gc_problem &p = g->p;
    Graph s;
    memset(&s, 0, sizeof(s));                  // padding too: views are compared bytewise
    const int cb = g->compact ? g->window_block : 0;
    s.W = p.width; s.H = p.height; s.J = (int32_t)stored_levels(&p, cb); s.Jf = p.labels - 1;
    s.plane = (int64_t)s.W * s.H;
    s.N = s.plane * s.J;
    char *b = (char *)g->ws;
    s.hdr = (GDEV DevHeader *)b; b += align256(sizeof(DevHeader));
    s.slots = (GDEV Slot *)b; b += align256(kSlots * sizeof(Slot));
    size_t w4 = align256((size_t)s.N * 4);
    GDEV int32_t **arr[] = {&s.ex, &s.ht, &s.rd, &s.re, &s.rs, &s.rem, &s.rep, &s.rsm, &s.rsp, &s.ein, &s.aux};
    for (GDEV int32_t **a : arr) { *a = (GDEV int32_t *)b; b += w4; }
    s.mask = (GDEV uint16_t *)b; b += align256((size_t)s.N * 2);
    s.wlo = (GDEV int32_t *)b; b += align256((size_t)s.plane * 4);
    s.whi = (GDEV int32_t *)b; b += align256((size_t)s.plane * 4);
    s.bact = (GDEV uint8_t *)b; b += align256(flag_bytes(s.N));
    s.binf = (GDEV uint8_t *)b; b += align256(flag_bytes(s.N));
    s.stamps = (GDEV int32_t *)b; b += align256(max_tiles(&p, cb) * 4);
    s.blist = (GDEV int32_t *)b; b += align256((size_t)((s.N + kBlock - 1) / kBlock) * 4);
    s.tlist = (GDEV int32_t *)b;
    s.te = 2 * p.penalty_h; s.ts = 2 * p.penalty_v;
    s.ie = p.inhibit_h; s.is = p.inhibit_v;
    s.win = g->window_block > 0 ? 1 : 0;
    s.cw = cb > 0 ? 1 : 0;
    return s;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

__device__ inline int wave_sum_i32(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ inline long long wave_sum_i64(long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ inline bool lane0() { return (threadIdx.x & 63) == 0; }

// Activity-flag group of this thread's wavefront in block lb.
__device__ inline int64_t group_of(int64_t lb) { return lb * (kBlock / kGroup) + (threadIdx.x >> 6); }

__device__ inline bool wave_any(bool p) { return __ballot(p) != 0; }

__device__ inline int wave_sum(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a kBlock-thread block; the result is valid in thread 0.  Every
// thread of the block must call it.
template <typename T>
__device__ inline T block_sum(T v)
{
    __shared__ T part[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane0()) part[threadIdx.x >> 6] = v;
    __syncthreads();
    T t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) t += part[i];
    return t;
}

__device__ inline Slot &my_slot(Slot *slots, int64_t lb) { return slots[lb & (kSlots - 1)]; }

// Maximum over a kBlock-thread block (non-negative values); valid in thread
// 0.  Every thread of the block must call it.
__device__ inline int block_max(int v)
{
    __shared__ int part[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_down(v, off, 64);
        v = o > v ? o : v;
    }
    if (lane0()) part[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) t = part[i] > t ? part[i] : t;
    return t;
}

// Kernel sources.  A solver kernel runs on one graph passed by value, one
// workgroup per 256 nodes or per tile, or over a device list of them.
constexpr int kMaxBatch = GC_BATCH_MAX_GRAPHS;
constexpr unsigned kGridX = 65535;      // x extent of a batch launch's 2-D grid

// 2-D grid holding `blocks` workgroups (x fastest).
inline dim3 batch_grid(int64_t blocks)
{
    if (blocks <= 0) blocks = 1;
    if (blocks <= kGridX) return dim3((unsigned)blocks, 1, 1);
    return dim3(kGridX, (unsigned)((blocks + kGridX - 1) / kGridX), 1);
}
// Phases of a member of a batch: the step a member takes next.
enum BatchPhase : int32_t {
    BP_INIT = 0, BP_SEED, BP_RELAX, BP_COUNT, BP_PUSH, BP_RELABEL, BP_SWEEP, BP_MERGE, BP_DONE
};

// Kinds of work unit, each run by its own launch so that each kernel keeps
// the register count of its own code: every block of the member (seeds,
// count, merge), a listed relaxation tile, a listed block of a sweep.
enum BatchKind : int32_t { BK_FULL = 0, BK_RELAX = 1, BK_SWEEP = 2 };

__host__ __device__ inline int batch_kind(int phase)
{
    return phase == BP_RELAX ? BK_RELAX
         : (phase == BP_PUSH || phase == BP_RELABEL || phase == BP_SWEEP) ? BK_SWEEP : BK_FULL;
}

// Device record of one member's progress through its solve.
struct MemberCtl {
    int32_t phase;            // phase of the current step
    int32_t pass;             // relaxation pass of the current global relabel, from 1
    int32_t sweep;            // sweeps done in the current period
    int32_t period;           // length of the current period
    int32_t round;            // global relabels begun
    int32_t status;           // GC_OK, or GC_E_NOT_CONVERGED when stopped at max_sweeps
    int32_t units;            // work units of the current step
    int32_t fused;            // fused sweeps (else push + relabel)
    int32_t blocks, tiles;    // 256-node blocks, relaxation tiles
    int32_t active, max_height;
    int32_t sweeps, passes, relabels;
    int32_t done_step;        // step in which it finished
    int32_t dense;            // this step's sweep takes every block in order (list too long)
    int32_t cut;              // 1: the current relabel stopped early; 2: it is being carried on
    long long pushes, visits;
};

// Device table of a batch.
struct BatchDev {
    int32_t ng;               // members in the table
    int32_t total[3];         // work units of the current step, per kind (BatchKind)
    int32_t live;             // members not finished
    int32_t step;             // steps run
    int32_t period, max_sweeps, local_iters, flags;
    int32_t relabel_passes;   // the option: > 0 a relabel's pass cap, < 0 none, 0 by depth
    int32_t pad[5];
    int32_t unit_off[3][kMaxBatch + 1];   // per kind, prefix of the members' units
    int32_t list_off[kMaxBatch + 1];   // prefix of the members' compaction workgroups
    MemberCtl ctl[kMaxBatch];
    Graph graphs[kMaxBatch];
};

// Runs f(graph, local block) for the block of a launch: one graph, the grid
// covering its blocks (or tiles) exactly.
template <class F>
__device__ inline void for_blocks(const Graph &s, int, F &&f)
{
    f(s, (int64_t)blockIdx.x);
}

// A list-driven launch over one graph: the workgroups of a fixed grid take
// the ids of a device list in turn (256-node blocks for the sweeps, tiles
// for a relaxation pass), so a launch costs its listed work and a grid of
// fixed size instead of one workgroup per block of the whole graph.
struct Listed {
    Graph s;
    const int32_t *ids;
    const int32_t *count;
};

template <class F>
__device__ inline void for_blocks(const Listed &L, int, F &&f)
{
    const int n = *L.count;
    // the id is the same in every lane: read it into a scalar register, so
    // that the block's index arithmetic and loads stay scalar
    for (int i = blockIdx.x; i < n; i += gridDim.x) f(L.s, (int64_t)__builtin_amdgcn_readfirstlane(L.ids[i]));
}

// Workgroup-wide compaction: every thread with `want` gets a distinct slot
// of ids[] (one atomic per workgroup on *count) and stores `id` there.
__device__ inline void block_append(bool want, int32_t id, int32_t *ids, int32_t *count)
{
    __shared__ int wave_n[kBlock / 64], base;
    const unsigned long long bal = __ballot(want);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wave_n[w] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < kBlock / 64; ++i) { const int c = wave_n[i]; wave_n[i] = t; t += c; }
        base = t ? atomicAdd(count, t) : 0;
    }
    __syncthreads();
    if (want) {
        const int rank = __popcll(bal & ((1ULL << lane) - 1ULL));
        ids[base + wave_n[w] + rank] = id;
    }
}

// Node counts stay below 2^29 (checked on the host), so 32-bit division is exact.
__device__ inline void decode(const Graph &s, int64_t n, int &j, int &y, int &x)
{
    const int n32 = (int)n, P = (int)s.plane;
    j = n32 / P;
    const int r = n32 - j * P;
    y = r / s.W;
    x = r - y * s.W;
}

__device__ inline int64_t nbr(const Graph &s, int64_t n, int d)
{
    return n + dir_dj(d) * s.plane + dir_dy(d) * (int64_t)s.W + dir_dx(d);
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Data term at every cross point (x, S, y).
__global__ void __launch_bounds__(kBlock)
k_cost_volume(const uint8_t *__restrict__ left, const uint8_t *__restrict__ right,
              int W, int H, int m, int cap, int32_t *__restrict__ cost)
{
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int y = blockIdx.y;
    int S = blockIdx.z;
    if (x >= W) return;
    int xl = x - S + (m - 1);
    int xr = x + S - (m - 1);
    int32_t g = cap;
    if (xl >= 0 && xl < W && xr >= 0 && xr < W) {
        int d = (int)left[(int64_t)y * W + xl] - (int)right[(int64_t)y * W + xr];
        d = d < 0 ? -d : d;
        g = d < cap ? d : cap;
    }
    cost[((int64_t)S * H + y) * W + x] = g;
}

// Colour data term (Sec. 4.3): sum over the three channels of the absolute
// differences, capped; images are [h][w][3] bytes.  Consecutive threads read
// consecutive 3-byte pixels, so a wave's loads stay within a few lines.
__global__ void __launch_bounds__(kBlock)
k_cost_volume_rgb(const uint8_t *__restrict__ left, const uint8_t *__restrict__ right,
                  int W, int H, int m, int cap, int32_t *__restrict__ cost)
{
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int y = blockIdx.y;
    int S = blockIdx.z;
    if (x >= W) return;
    int xl = x - S + (m - 1);
    int xr = x + S - (m - 1);
    int32_t g = cap;
    if (xl >= 0 && xl < W && xr >= 0 && xr < W) {
        const uint8_t *a = left + ((int64_t)y * W + xl) * 3;
        const uint8_t *b = right + ((int64_t)y * W + xr) * 3;
        int sad = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int d = (int)a[c] - (int)b[c];
            sad += d < 0 ? -d : d;
        }
        g = sad < cap ? sad : cap;
    }
    cost[((int64_t)S * H + y) * W + x] = g;
}

// Node classes of a thin-skin graph: a level inside the site's window is
// free; levels at or above its top are forced to the source side, levels
// below its bottom to the sink side.
enum NodeClass { FREE = 0, FSRC = 1, FSNK = 2 };
__device__ inline int node_class(int k, int lo, int hi) { return k <= lo ? FSRC : k > hi ? FSNK : FREE; }

// Which of the 14 arcs of node (j, y, x) exist, as a bit mask over Dir.
__device__ inline unsigned arc_exists(const Graph &s, int j, int y, int x)
{
    const bool hE = x + 1 < s.W, hW = x > 0, hS = y + 1 < s.H, hN = y > 0;
    const bool hU = j > 0, hD = j + 1 < s.Jf;
    return (unsigned)hD << D_DOWN | (unsigned)hU << D_UP | (unsigned)hE << D_E |
           (unsigned)hW << D_W | (unsigned)hS << D_S | (unsigned)hN << D_N |
           (unsigned)(hE && hU) << D_EM | (unsigned)(hE && hD) << D_EP |
           (unsigned)(hW && hU) << D_WM | (unsigned)(hW && hD) << D_WP |
           (unsigned)(hS && hU) << D_SM | (unsigned)(hS && hD) << D_SP |
           (unsigned)(hN && hU) << D_NM | (unsigned)(hN && hD) << D_NP;
}

// The stored pair word of the arc of node n in direction d.  For the
// directions whose word lives at n the word is the out-residual; for the
// others it is the residual of the opposite arc.
__device__ inline int32_t *word_ptr(const Graph &s, int64_t n, int d)
{
    const int64_t P = s.plane, W = s.W;
    switch (d) {
    case D_DOWN: return s.rd + n;
    case D_UP:   return s.rd + (n - P);
    case D_E:    return s.re + n;
    case D_W:    return s.re + (n - 1);
    case D_S:    return s.rs + n;
    case D_N:    return s.rs + (n - W);
    case D_EM:   return s.rem + n;
    case D_EP:   return s.rep + n;
    case D_WM:   return s.rep + (n - P - 1);
    case D_WP:   return s.rem + (n + P - 1);
    case D_SM:   return s.rsm + n;
    case D_SP:   return s.rsp + n;
    case D_NM:   return s.rsp + (n - P - W);
    default:     return s.rsm + (n + P - W);       // D_NP
    }
}

__host__ __device__ constexpr bool word_is_forward(int d)
{
    return d == D_DOWN || d == D_E || d == D_S || d == D_EM || d == D_EP || d == D_SM || d == D_SP;
}

// Out-residual from the stored word.
__device__ inline int32_t res_from_word(const Graph &s, int d, int32_t w)
{
    if (word_is_forward(d)) return w;
    switch (d) {
    case D_UP: return kInf;
    case D_W:  return s.te - w;
    case D_N:  return s.ts - w;
    case D_WM: case D_WP: return s.ie - w;
    default:   return s.is - w;                        // D_NM, D_NP
    }
}

// Residual of the in-arc into n from its neighbour in direction d, from the
// pair word of that arc.
__device__ inline int32_t in_res_from_word(const Graph &s, int d, int32_t w)
{
    switch (d) {
    case D_DOWN: return kInf;                           // v_{k+1} -> v_k
    case D_E:    return s.te - w;
    case D_S:    return s.ts - w;
    case D_EM: case D_EP: return s.ie - w;
    case D_SM: case D_SP: return s.is - w;
    default:     return w;                              // word holds the in-residual
    }
}

// Word and partner height of arc d of node n, read without a branch: for a
// missing arc (ok false) both read node n's own height, an in-bounds address
// whose value the caller ignores.  With unconditional loads the compiler
// issues all of a node's loads before the first wait; loads under per-arc
// branches were issued and awaited one arc at a time.
__device__ inline int32_t load_word(const Graph &s, int64_t n, int d, bool ok)
{
    return *(ok ? word_ptr(s, n, d) : s.ht + n);
}

__device__ inline int32_t load_height(const Graph &s, int64_t n, int d, bool ok)
{
    return s.ht[ok ? nbr(s, n, d) : n];
}

// The array holding the pair word of arc direction d: the node's own entry
// for the forward directions, the neighbour's for the others.
__device__ inline int32_t *word_array(const Graph &s, int d)
{
    switch (d) {
    case D_DOWN: case D_UP: return s.rd;
    case D_E: case D_W:     return s.re;
    case D_S: case D_N:     return s.rs;
    case D_EM: case D_WP:   return s.rem;
    case D_EP: case D_WM:   return s.rep;
    case D_SM: case D_NP:   return s.rsm;
    default:                return s.rsp;          // D_SP, D_NM
    }
}

// Arc topology of a node, for the kernels shared by full graphs and compact
// thin skins.  ex: the node's existing arcs; nb: the neighbour's index;
// wp: the arc's pair word.
//
// Full graph (or a skin in the full layout): the 14 lattice arcs.
struct FullTopo {
    unsigned ex;
    __device__ FullTopo(const Graph &s, int64_t, int j, int y, int x) : ex(arc_exists(s, j, y, x)) {}
    __device__ int64_t nb(const Graph &s, int64_t n, int d) const { return nbr(s, n, d); }
    __device__ int32_t *wp(const Graph &s, int64_t n, int d) const { return word_ptr(s, n, d); }
};

// Compact thin skin: stored level t of site (x, y) is level wlo + t, for
// t < whi - wlo (higher stored levels are padding, with no arcs).  A
// neighbour across a site boundary at level offset dj therefore sits
// dj + wlo(own) - wlo(other) stored levels away, and the arc exists only when
// that level is inside the other site's window; arcs to levels outside it
// (forced nodes) were folded into the node's excess when the skin was built.
struct SkinTopo {
    unsigned ex;
    int dl[4];                  // wlo(own) - wlo(E, W, S, N)
    __device__ SkinTopo(const Graph &s, int64_t, int t, int y, int x)
    {
        const int64_t site = (int64_t)y * s.W + x;
        const int lo = s.wlo[site], len = s.whi[site] - lo;
        ex = 0;
        dl[0] = dl[1] = dl[2] = dl[3] = 0;
        if (t >= len) return;                              // padding level
        unsigned m = (t + 1 < len ? 1u << D_DOWN : 0u) | (t > 0 ? 1u << D_UP : 0u);
        auto side = [&](bool in, int64_t other, int i, int d0, int dm, int dp) {
            if (!in) return;
            const int lo2 = s.wlo[other], len2 = s.whi[other] - lo2;
            const int tt = t + lo - lo2;                    // same level at the other site
            dl[i] = lo - lo2;
            m |= (tt >= 0 && tt < len2 ? 1u << d0 : 0u) | (tt >= 1 && tt - 1 < len2 ? 1u << dm : 0u) |
                 (tt + 1 >= 0 && tt + 1 < len2 ? 1u << dp : 0u);
        };
        side(x + 1 < s.W, site + 1, 0, D_E, D_EM, D_EP);
        side(x > 0, site - 1, 1, D_W, D_WM, D_WP);
        side(y + 1 < s.H, site + s.W, 2, D_S, D_SM, D_SP);
        side(y > 0, site - s.W, 3, D_N, D_NM, D_NP);
        ex = m;
    }
    __device__ int shift(int d) const
    {
        return dir_dx(d) > 0 ? dl[0] : dir_dx(d) < 0 ? dl[1] : dir_dy(d) > 0 ? dl[2] : dir_dy(d) < 0 ? dl[3] : 0;
    }
    __device__ int64_t nb(const Graph &s, int64_t n, int d) const
    {
        return n + (dir_dj(d) + shift(d)) * s.plane + dir_dy(d) * (int64_t)s.W + dir_dx(d);
    }
    __device__ int32_t *wp(const Graph &s, int64_t n, int d) const
    {
        return word_array(s, d) + (word_is_forward(d) ? n : nb(s, n, d));
    }
};

template <class T>
__device__ inline int32_t load_word(const Graph &s, const T &tp, int64_t n, int d, bool ok)
{
    return *(ok ? tp.wp(s, n, d) : s.ht + n);
}

template <class T>
__device__ inline int32_t load_height(const Graph &s, const T &tp, int64_t n, int d, bool ok)
{
    return s.ht[ok ? tp.nb(s, n, d) : n];
}

// Capacities of the arc from node (j, site) to its neighbour in direction d
// (cout) and of the arc back (cin), Sec. 3 / Fig. 4: data chain g(k) down,
// same-level penalty both ways, inhibit on u_{k+1} -> v_k.  The unbounded
// chain reverse is reported as 0: it never meets a forced partner of a free
// node, and a forced node only uses the capacity towards a free one.
__device__ inline void arc_caps(const Graph &s, const int32_t *__restrict__ cost, int d, int64_t site,
                                int j, int ph, int pv, int32_t &cout, int32_t &cin)
{
    cout = 0;
    cin = 0;
    switch (d) {
    case D_DOWN: cout = cost[(int64_t)(j + 1) * s.plane + site]; break;
    case D_UP:   cin = cost[(int64_t)j * s.plane + site]; break;
    case D_E: case D_W: cout = cin = ph; break;
    case D_S: case D_N: cout = cin = pv; break;
    case D_EM: case D_WM: cout = s.ie; break;
    case D_EP: case D_WP: cin = s.ie; break;
    case D_SM: case D_NM: cout = s.is; break;
    default: cin = s.is; break;                  // D_SP, D_NP
    }
}

// Graph initialisation.  Terminal arcs are folded into node overflows: the
// arc from s into v_1 is pre-saturated (excess g(0)) and the arc from
// v_{m-1} to t becomes a deficit g(m-1).  For a thin-skin graph (kWindow) the
// same folding applies to every arc between a free node and a forced one:
// arcs from forced-source nodes are pre-saturated into the free node's
// excess, arcs into forced-sink nodes become deficits, and forced nodes are
// inert (no excess, infinite height, no residual arc from a free node into
// them).  tcap sums the sink-side capacity, c0 the capacity of arcs running
// straight from forced-source to forced-sink nodes (cut by every labelling).
template <bool kWindow>
__global__ void __launch_bounds__(kBlock)
k_build(Graph s, const int32_t *__restrict__ cost, int m, int cap)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    long long tsum = 0, c0 = 0;
    if (n < s.N) {
        int j, y, x;
        decode(s, n, j, y, x);
        const int64_t site = (int64_t)y * s.W + x;
        const int k = j + 1;
        // the int32 bounds on flow and excess assume every data term lies in
        // [0, cap]: node j checks cost layer j + 1, the first layer also layer 0
        const int32_t ck = cost[(int64_t)k * s.plane + site];
        const int32_t c0v = j == 0 ? cost[site] : 0;
        if (ck < 0 || ck > cap || c0v < 0 || c0v > cap) atomicOr(&s.hdr->prefix_err, kCostErr);
        const bool hasE = x + 1 < s.W, hasS = y + 1 < s.H;
        if (!kWindow) {
            int32_t e = 0;
            if (k == 1) e += cost[site];                                    // s -> v_1
            if (k == m - 1) {                                                // v_{m-1} -> t
                const int32_t gt = cost[(int64_t)(m - 1) * s.plane + site];
                e -= gt;
                tsum = gt;
            }
            s.ex[n] = e;
            s.ht[n] = 0;
            s.ein[n] = 0;
            s.rd[n] = (j + 1 < s.J) ? cost[(int64_t)k * s.plane + site] : 0;
            s.re[n] = hasE ? s.te / 2 : 0;
            s.rs[n] = hasS ? s.ts / 2 : 0;
            s.rem[n] = (hasE && j > 0) ? s.ie : 0;      // v_k -> E_{k-1} carries the capacity
            s.rep[n] = 0;                               // its capacity runs E_{k+1} -> v_k
            s.rsm[n] = (hasS && j > 0) ? s.is : 0;
            s.rsp[n] = 0;
        } else {
            const int lo = s.wlo[site], hi = s.whi[site];
            const int cn = node_class(k, lo, hi);
            const unsigned ex_mask = arc_exists(s, j, y, x);
            const int ph = s.te / 2, pv = s.ts / 2;
            int32_t e = 0;
#pragma unroll
            for (int d = 0; d < 14; ++d) {
                if (!((ex_mask >> d) & 1u)) continue;
                const int dx = dir_dx(d), dy = dir_dy(d);
                const int64_t psite = site + dy * (int64_t)s.W + dx;
                const int cp = (dx == 0 && dy == 0) ? node_class(k + dir_dj(d), lo, hi)
                                                    : node_class(k + dir_dj(d), s.wlo[psite], s.whi[psite]);
                int32_t cout, cin;
                arc_caps(s, cost, d, site, j, ph, pv, cout, cin);
                if (cn == FREE) {
                    if (cp == FSRC) e += cin;
                    else if (cp == FSNK) { e -= cout; tsum += cout; }
                } else if (cn == FSRC && cp == FSNK) {
                    c0 += cout;
                }
                if (word_is_forward(d)) {
                    int32_t wd = 0;
                    if (cn == FREE) wd = cp == FREE ? cout : cp == FSRC ? cout + cin : 0;
                    else if (cn == FSNK && cp == FREE) wd = cout + cin;
                    *word_ptr(s, n, d) = wd;
                }
            }
            if (!((ex_mask >> D_DOWN) & 1u)) s.rd[n] = 0;
            if (!((ex_mask >> D_E) & 1u)) s.re[n] = 0;
            if (!((ex_mask >> D_S) & 1u)) s.rs[n] = 0;
            if (!((ex_mask >> D_EM) & 1u)) s.rem[n] = 0;
            if (!((ex_mask >> D_EP) & 1u)) s.rep[n] = 0;
            if (!((ex_mask >> D_SM) & 1u)) s.rsm[n] = 0;
            if (!((ex_mask >> D_SP) & 1u)) s.rsp[n] = 0;
            if (cn == FREE) {
                if (j == 0) e += cost[site];                                  // from s
                if (j + 1 == s.J) {                                           // into t
                    const int32_t gt = cost[(int64_t)(m - 1) * s.plane + site];
                    e -= gt;
                    tsum += gt;
                }
            }
            s.ex[n] = cn == FREE ? e : 0;
            s.ht[n] = cn == FREE ? 0 : kInf;
            s.ein[n] = 0;
        }
    }
    tsum = block_sum(tsum);
    __syncthreads();
    c0 = block_sum(c0);
    if (threadIdx.x == 0) {
        if (tsum) atomicAdd((unsigned long long *)&my_slot(s.slots, blockIdx.x).tcap, (unsigned long long)tsum);
        if (c0) atomicAdd((unsigned long long *)&my_slot(s.slots, blockIdx.x).c0, (unsigned long long)c0);
    }
}

// Compact thin-skin initialisation: one thread per stored node.  A free
// level gets what k_build<true> gives it (terminal arcs and arcs to forced
// nodes folded into its overflow, forced neighbours absent); a padding level
// is inert.  The data terms the skin reads (layers j and j + 1 of each free
// level j) are checked against [0, cap].
__global__ void __launch_bounds__(kBlock)
k_build_skin(Graph s, const int32_t *__restrict__ cost, int m, int cap)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    long long tsum = 0;
    if (n < s.N) {
        int t, y, x;
        decode(s, n, t, y, x);
        const int64_t site = (int64_t)y * s.W + x;
        const int lo = s.wlo[site], hi = s.whi[site];
        int32_t *const words[7] = {s.rd, s.re, s.rs, s.rem, s.rep, s.rsm, s.rsp};
        if (t >= hi - lo) {
            s.ex[n] = 0;
            s.ht[n] = kInf;
            s.ein[n] = 0;
#pragma unroll
            for (int i = 0; i < 7; ++i) words[i][n] = 0;
        } else {
            const int j = lo + t, k = j + 1;
            const int32_t ca = cost[(int64_t)j * s.plane + site], cb = cost[(int64_t)k * s.plane + site];
            if (ca < 0 || ca > cap || cb < 0 || cb > cap) atomicOr(&s.hdr->prefix_err, kCostErr);
            const unsigned ex_mask = arc_exists(s, j, y, x);
            const int ph = s.te / 2, pv = s.ts / 2;
            int32_t e = 0;
#pragma unroll
            for (int i = 0; i < 7; ++i) words[i][n] = 0;
#pragma unroll
            for (int d = 0; d < 14; ++d) {
                if (!((ex_mask >> d) & 1u)) continue;
                const int dx = dir_dx(d), dy = dir_dy(d);
                const int64_t psite = site + dy * (int64_t)s.W + dx;
                const int cp = (dx == 0 && dy == 0) ? node_class(k + dir_dj(d), lo, hi)
                                                    : node_class(k + dir_dj(d), s.wlo[psite], s.whi[psite]);
                int32_t cout, cin;
                arc_caps(s, cost, d, site, j, ph, pv, cout, cin);
                if (cp == FSRC) e += cin;
                else if (cp == FSNK) { e -= cout; tsum += cout; }
                if (word_is_forward(d))
                    word_array(s, d)[n] = cp == FREE ? cout : cp == FSRC ? cout + cin : 0;
            }
            if (j == 0) e += cost[site];                                      // from s
            if (j + 1 == s.Jf) {                                              // into t
                const int32_t gt = cost[(int64_t)(m - 1) * s.plane + site];
                e -= gt;
                tsum += gt;
            }
            s.ex[n] = e;
            s.ht[n] = 0;
            s.ein[n] = 0;
        }
    }
    tsum = block_sum(tsum);
    if (threadIdx.x == 0 && tsum)
        atomicAdd((unsigned long long *)&my_slot(s.slots, blockIdx.x).tcap, (unsigned long long)tsum);
}

// Capacity of the arcs from forced-source to forced-sink nodes of a compact
// skin, which stores neither: one thread per site sums, for each arc
// direction to a neighbouring site, the levels k <= wlo(own) whose partner
// level k + dj lies above the neighbour's window (k + dj > whi), times the
// arc's capacity (constant along the column for lateral arcs; within a
// column no such arc exists, the window holding at least one level).
__global__ void __launch_bounds__(kBlock)
k_skin_c0(Graph s, int m)
{
    const int64_t site = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    long long c0 = 0;
    if (site < s.plane) {
        const int y = (int)(site / s.W), x = (int)(site - (int64_t)y * s.W);
        const int lo = s.wlo[site];
        const int ph = s.te / 2, pv = s.ts / 2;
#pragma unroll
        for (int d = D_E; d < 14; ++d) {
            const int dx = dir_dx(d), dy = dir_dy(d), dj = dir_dj(d);
            const int nx = x + dx, ny = y + dy;
            if (nx < 0 || nx >= s.W || ny < 0 || ny >= s.H) continue;
            int32_t cout, cin;
            arc_caps(s, nullptr, d, site, 0, ph, pv, cout, cin);
            if (cout == 0) continue;
            const int hi2 = s.whi[(int64_t)ny * s.W + nx];
            int a = 1 > 1 - dj ? 1 : 1 - dj;                 // k and k + dj are levels 1 .. m-1
            a = a > hi2 + 1 - dj ? a : hi2 + 1 - dj;         // k + dj > whi(other)
            int z = lo < m - 1 ? lo : m - 1;                 // k <= wlo(own)
            z = z < m - 1 - dj ? z : m - 1 - dj;
            if (z >= a) c0 += (long long)cout * (z - a + 1);
        }
    }
    c0 = block_sum(c0);
    if (threadIdx.x == 0 && c0)
        atomicAdd((unsigned long long *)&my_slot(s.slots, blockIdx.x).c0, (unsigned long long)c0);
}

// Thin-skin windows from the delegate-point labels (Sec. 4.5): the labels of
// the coarse group and of the groups directly above and below.
__global__ void __launch_bounds__(kBlock)
k_windows(Graph s, const int32_t *__restrict__ coarse_labels, int b, int m)
{
    int64_t site = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (site >= s.plane) return;
    const int y = (int)(site / s.W), x = (int)(site - (int64_t)y * s.W);
    const int wc = (s.W + b - 1) / b;
    const int Sc = coarse_labels[(int64_t)(y / b) * wc + x / b];
    const int lo = b * (Sc - 1), hi = b * (Sc + 2) - 1;
    s.wlo[site] = lo < 0 ? 0 : lo;
    s.whi[site] = hi > m - 1 ? m - 1 : hi;
}

// Delegate-point data term: the sum over the b x b sites of a coarse site of
// the cheapest label in the coarse label group.
__global__ void __launch_bounds__(kBlock)
k_coarse_cost(const int32_t *__restrict__ cost, int W, int H, int m, int b,
              int32_t *__restrict__ coarse)
{
    const int wc = (W + b - 1) / b, hc = (H + b - 1) / b;
    const int X = blockIdx.x * blockDim.x + threadIdx.x;
    const int Y = blockIdx.y, Sc = blockIdx.z;
    if (X >= wc) return;
    const int64_t plane = (int64_t)W * H;
    int32_t sum = 0;
    for (int y = Y * b; y < Y * b + b && y < H; ++y)
        for (int x = X * b; x < X * b + b && x < W; ++x) {
            int32_t best = 0x7fffffff;
            for (int S = Sc * b; S < Sc * b + b && S < m; ++S) {
                const int32_t g = cost[(int64_t)S * plane + (int64_t)y * W + x];
                best = g < best ? g : best;
            }
            sum += best;
        }
    coarse[((int64_t)Sc * hc + Y) * wc + X] = sum;
}

// Push sweep.  The 14 neighbour heights of an active node are loaded first;
// only arcs to a neighbour exactly one below are admissible, so only their
// words are loaded next (a second round of memory latency that saves most
// word loads).  Pushes then run in registers and write the new words
// directly.
template <class T = FullTopo>
__device__ inline void push_blk(const Graph &s, int64_t lb)
{
    const int64_t g = group_of(lb);
    if (!s.bact[g]) return;                   // no active node in this wavefront's group
    int64_t n = lb * kBlock + threadIdx.x;
    int cnt = 0, vis = 0;
    if (n < s.N) {
        int32_t e = s.ex[n];
        const int32_t h = s.ht[n];
        if (e > 0 && h < kInf) {
            vis = 1;
            int j, y, x;
            decode(s, n, j, y, x);
            const T tp(s, n, j, y, x);
            const unsigned ex_mask = tp.ex;
            unsigned cand = 0;                // existing arcs to height h - 1
#pragma unroll
            for (int d = 0; d < 14; ++d) {
                const bool ok = (ex_mask >> d) & 1u;
                const int32_t hv = ok ? s.ht[tp.nb(s, n, d)] : kInf;
                cand |= (hv == h - 1 ? 1u : 0u) << d;
            }
            int32_t w[14];
#pragma unroll
            for (int d = 0; d < 14; ++d)
                w[d] = ((cand >> d) & 1u) ? *tp.wp(s, n, d) : 0;
#pragma unroll
            for (int d = 0; d < 14; ++d) {
                if (!((cand >> d) & 1u)) continue;
                const int32_t r = res_from_word(s, d, w[d]);
                if (e > 0 && r > 0) {
                    const int32_t delta = e < r ? e : r;
                    *tp.wp(s, n, d) = word_is_forward(d) ? w[d] - delta : w[d] + delta;
                    const int64_t v = tp.nb(s, n, d);
                    atomicAdd(&s.ein[v], delta);
                    s.binf[v / kGroup] = 1;
                    e -= delta;
                    ++cnt;
                }
            }
            s.ex[n] = e;
        }
    }
    cnt = wave_sum(cnt);                      // no barrier: the wavefront finishes alone
    vis = wave_sum(vis);
    if (lane0() && cnt) atomicAdd(&my_slot(s.slots, g).pushes, (unsigned long long)cnt);
    if (lane0() && vis) atomicAdd(&my_slot(s.slots, g).visits, (unsigned long long)vis);
}

template <class Src, class T = FullTopo>
__global__ void __launch_bounds__(kBlock)
k_push(Src src)
{
    for_blocks(src, 0, [&](const Graph &s, int64_t lb) { push_blk<T>(s, lb); });
}

// Relabel sweep: merges the inflow of the push sweep, then lifts every
// active node to one above its lowest residual neighbour.
template <class T = FullTopo>
__device__ inline void relabel_blk(const Graph &s, int64_t lb)
{
    // Loads that do not depend on each other are written before the first
    // use or store, so they go out together (the compiler cannot move a load
    // above a store to another of the state arrays: they might alias).
    const int64_t g = group_of(lb);
    const uint8_t was_active = s.bact[g], got_inflow = s.binf[g];
    if (!was_active && !got_inflow) return;   // nothing arrived, nothing to lift
    int64_t n = lb * kBlock + threadIdx.x;
    bool active = false;
    if (n < s.N) {
        const int32_t in = s.ein[n];
        const int32_t e = s.ex[n] + in;
        const int32_t h = s.ht[n];
        if (e > 0 && h < kInf) {
            int j, y, x;
            decode(s, n, j, y, x);
            const T tp(s, n, j, y, x);
            const unsigned ex_mask = tp.ex;
            int32_t w[14], hv[14];
#pragma unroll
            for (int d = 0; d < 14; ++d) {
                const bool ok = (ex_mask >> d) & 1u;
                w[d] = load_word(s, tp, n, d, ok);
                hv[d] = load_height(s, tp, n, d, ok);
            }
            int32_t hmin = kInf;
#pragma unroll
            for (int d = 0; d < 14; ++d)
                if (((ex_mask >> d) & 1u) && res_from_word(s, d, w[d]) > 0)
                    hmin = hv[d] < hmin ? hv[d] : hmin;
            const int32_t nh = hmin >= kInf ? kInf : hmin + 1;
            if (nh > h) s.ht[n] = nh;
            active = nh < kInf;
        }
        if (in != 0) {                        // stores last: no load waits behind them
            s.ex[n] = e;
            s.ein[n] = 0;
        }
    }
    const bool any = wave_any(active);        // no barrier: the wavefront finishes alone
    if (lane0()) {
        if (any != (was_active != 0)) s.bact[g] = any;
        if (got_inflow) s.binf[g] = 0;
    }
}

template <class Src, class T = FullTopo>
__global__ void __launch_bounds__(kBlock)
k_relabel(Src src)
{
    for_blocks(src, 0, [&](const Graph &s, int64_t lb) { relabel_blk<T>(s, lb); });
}

// Fused sweep: one kernel per push-relabel step.  Every node of a 64-node
// group that holds an active node or received inflow merges its inflow, relabels
// to one above its lowest residual neighbour when no neighbour is lower, and
// pushes along residual arcs to lower neighbours.  Neighbour heights are
// read while they change; a stale height is never above the current one
// (heights only grow between global relabels), and the two nodes of an arc
// pair move flow in opposite directions, so with atomic updates of the pair
// word every residual stays within [0, pair total] whatever the order.  The
// labelling may lose validity between global relabels; only the exact global
// relabel decides termination, so the final state is the same max preflow.
template <class T = FullTopo>
__device__ inline void sweep_blk(const Graph &s, int64_t lb)
{
    const int64_t g = group_of(lb);
    const uint8_t inflow = s.binf[g], was_active = s.bact[g];
    if (!inflow && !was_active) return;
    // The flag is cleared before the inflow is merged.  A push landing in
    // between may still lose its flag (neither side waits for its stores);
    // its inflow then waits in ein for a later flag or for k_merge, which
    // ends every period by merging every node.
    if (inflow && lane0()) s.binf[g] = 0;
    const int64_t n = lb * kBlock + threadIdx.x;
    bool active = false;
    int cnt = 0, vis = 0;
    if (n < s.N) {
        int32_t e = s.ex[n];
        const int32_t in = s.ein[n];
        int32_t h = s.ht[n];                      // loaded with ex and ein, before the exchange
        const int32_t e0 = e;
        if (in != 0) e += atomicExch(&s.ein[n], 0);
        if (e > 0 && h < kInf) {
            vis = 1;
            int j, y, x;
            decode(s, n, j, y, x);
            const T tp(s, n, j, y, x);
            const unsigned ex_mask = tp.ex;
            int32_t r[14], hv[14];
#pragma unroll
            for (int d = 0; d < 14; ++d) {
                const bool ok = (ex_mask >> d) & 1u;
                r[d] = load_word(s, tp, n, d, ok);
                hv[d] = load_height(s, tp, n, d, ok);
            }
#pragma unroll
            for (int d = 0; d < 14; ++d) {       // after all loads are issued
                const bool ok = (ex_mask >> d) & 1u;
                r[d] = ok ? res_from_word(s, d, r[d]) : 0;
                hv[d] = ok ? hv[d] : kInf;
            }
            int32_t hmin = kInf;
#pragma unroll
            for (int d = 0; d < 14; ++d)
                if (r[d] > 0) hmin = hv[d] < hmin ? hv[d] : hmin;
            if (hmin >= h) {                       // no lower neighbour: relabel
                h = hmin >= kInf ? kInf : hmin + 1;
                s.ht[n] = h;
            }
#pragma unroll
            for (int d = 0; d < 14; ++d) {
                if (e > 0 && r[d] > 0 && hv[d] < h) {
                    const int32_t delta = e < r[d] ? e : r[d];
                    atomicAdd(tp.wp(s, n, d), word_is_forward(d) ? -delta : delta);
                    const int64_t v = tp.nb(s, n, d);
                    atomicAdd(&s.ein[v], delta);
                    s.binf[v / kGroup] = 1;
                    e -= delta;
                    ++cnt;
                }
            }
            active = e > 0 && h < kInf;
        }
        if (e != e0) s.ex[n] = e;
    }
    const bool any = wave_any(active);        // no barrier: the wavefront finishes alone
    cnt = wave_sum(cnt);
    vis = wave_sum(vis);
    if (lane0()) {
        if (any != (was_active != 0)) s.bact[g] = any;
        if (cnt) atomicAdd(&my_slot(s.slots, g).pushes, (unsigned long long)cnt);
        if (vis) atomicAdd(&my_slot(s.slots, g).visits, (unsigned long long)vis);
    }
}

template <class Src, class T = FullTopo>
__global__ void __launch_bounds__(kBlock)
k_sweep(Src src)
{
    for_blocks(src, 0, [&](const Graph &s, int64_t lb) { sweep_blk<T>(s, lb); });
}

// Merges the inflow left by the last fused sweep into the excess.  Every
// node is visited: a group's inflow flag is cleared and set by different
// wavefronts of one sweep without ordering, so it may read 0 while inflow is
// pending.
__device__ inline void merge_blk(const Graph &s, int64_t lb)
{
    const int64_t n = lb * kBlock + threadIdx.x;
    if (n >= s.N) return;
    const int32_t in = s.ein[n];
    if (in != 0) {
        s.ex[n] += in;
        s.ein[n] = 0;
    }
}

template <class Src>
__global__ void __launch_bounds__(kBlock)
k_merge(Src src)
{
    for_blocks(src, 0, [&](const Graph &s, int64_t lb) { merge_blk(s, lb); });
}

// Work list of the next sweep: the 256-node blocks that hold a group with an
// active node (which 1: push sweeps) or with an active node or inflow
// (which 0: fused and relabel sweeps).  The list's length is counted in
// lists[par], and lists[par ^ 1] is cleared for the next list, whose
// previous reader has finished (launches on one stream run in order).
__global__ void __launch_bounds__(kBlock)
k_list_blocks(Graph s, int par, int which)
{
    const int64_t lb = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const int64_t nb = (s.N + kBlock - 1) / kBlock;
    bool want = false;
    if (lb < nb) {
        const uint32_t a = *(const uint32_t *)(s.bact + 4 * lb);
        const uint32_t f = which == 0 ? *(const uint32_t *)(s.binf + 4 * lb) : 0u;
        want = (a | f) != 0u;
    }
    block_append(want, (int32_t)lb, s.blist, &s.hdr->lists[par]);
    if (blockIdx.x == 0 && threadIdx.x == 0) s.hdr->lists[par ^ 1] = 0;
}

// Work list of relaxation pass `pass`: every tile in pass 1, afterwards the
// tiles with a tile of their 3x3x3 neighbourhood changed in the pass before
// (the test k_relax makes for itself).  Counted in lists[2 + par].
__global__ void __launch_bounds__(kBlock)
k_list_tiles(Graph s, int pass, int par, int tw, int th, int tj)
{
    const int ntx = (s.W + tw - 1) / tw, nty = (s.H + th - 1) / th, ntz = (s.J + tj - 1) / tj;
    const int64_t nt = (int64_t)ntx * nty * ntz;
    const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    bool want = false;
    if (t < nt) {
        if (pass == 1) {
            want = true;
        } else {
            const int bx = (int)(t % ntx), by = (int)((t / ntx) % nty), bz = (int)(t / ((int64_t)ntx * nty));
            for (int q = 0; q < 27 && !want; ++q) {
                const int tz = bz + q / 9 - 1, ty = by + (q / 3) % 3 - 1, tx = bx + q % 3 - 1;
                if (tz >= 0 && tz < ntz && ty >= 0 && ty < nty && tx >= 0 && tx < ntx)
                    want = (s.stamps[(tz * nty + ty) * ntx + tx] >> 1) == pass - 1;
            }
        }
    }
    block_append(want, (int32_t)t, s.tlist, &s.hdr->lists[2 + par]);
    if (blockIdx.x == 0 && threadIdx.x == 0) s.hdr->lists[2 + (par ^ 1)] = 0;
}

__device__ inline bool is_frozen(const Graph &s, int j, int y, int x)
{
    const int64_t site = (int64_t)y * s.W + x;
    return node_class(j + 1, s.wlo[site], s.whi[site]) != FREE;
}

// mode 0: out-arc mask (distance to deficits); mode 1: in-arc mask
// (reachability from excess).  Forced nodes of a thin-skin graph get no
// arcs, so relaxation never gives them a finite value.
template <class T = FullTopo>
__device__ inline void mask_blk(const Graph &s, int64_t lb, int mode)
{
    int64_t n = lb * kBlock + threadIdx.x;
    if (n >= s.N) return;
    int j, y, x;
    decode(s, n, j, y, x);
    if (s.win && !s.cw && is_frozen(s, j, y, x)) { s.mask[n] = 0; return; }
    const T tp(s, n, j, y, x);
    const unsigned ex_mask = tp.ex;
    int32_t w[14];
#pragma unroll
    for (int d = 0; d < 14; ++d) w[d] = load_word(s, tp, n, d, (ex_mask >> d) & 1u);
    unsigned mk = 0;
#pragma unroll
    for (int d = 0; d < 14; ++d) {
        const int32_t r = mode == 0 ? res_from_word(s, d, w[d]) : in_res_from_word(s, d, w[d]);
        mk |= (((ex_mask >> d) & 1u) && r > 0 ? 1u : 0u) << d;
    }
    s.mask[n] = (uint16_t)mk;
}

template <class Src, class T = FullTopo>
__global__ void __launch_bounds__(kBlock)
k_mask(Src src, int mode)
{
    for_blocks(src, 0, [&](const Graph &s, int64_t lb) { mask_blk<T>(s, lb, mode); });
}

// Seeds: mode 0 -> ht = 1 at deficit nodes, INF elsewhere;
//        mode 1 -> aux = 0 at excess nodes, INF elsewhere.
__device__ inline void seed_blk(const Graph &s, int64_t lb, int mode)
{
    int64_t n = lb * kBlock + threadIdx.x;
    if (n >= s.N) return;
    int32_t e = s.ex[n];
    if (s.win && !s.cw) {                     // (a compact skin stores free levels only)
        int j, y, x;
        decode(s, n, j, y, x);
        if (is_frozen(s, j, y, x)) e = 0;          // inert: never a seed
    }
    if (mode == 0) s.ht[n] = e < 0 ? 1 : kInf;
    else s.aux[n] = e > 0 ? 0 : kInf;
}

template <class Src>
__global__ void __launch_bounds__(kBlock)
k_seed(Src src, int mode)
{
    for_blocks(src, 0, [&](const Graph &s, int64_t lb) { seed_blk(s, lb, mode); });
}

// One tiled min-plus relaxation pass: val(u) = min(val(u), val(w) + step)
// over the neighbours w selected by mask(u).  Values only decrease, so
// tiles may run in any order and read each other's halos while they change;
// the pass sequence converges to the exact fixpoint.
//
// Across tiles, work is skipped: stamps[t] = 2*pass + u records the last
// pass in which tile t changed (u = 1 if it stopped before its local
// fixpoint), and in pass p > 1 a tile runs only if a tile of its 3x3x3
// neighbourhood (itself included) changed in pass p-1.  Inside the tile,
// every round re-evaluates all nodes in place in LDS (values written in a
// round are seen by later reads of the same round, which only speeds
// convergence) and one barrier-with-OR ends the rounds when none changed, at
// most max_rounds of them.  (A worklist of woken nodes with LDS atomics did
// less arithmetic but measured 30 % slower: the rounds are bound by barrier
// and LDS latency, not by the evaluations.)  flags[p % kMaxFlags] <- 1 if
// any value changed; pass p returns at once when pass p-1 changed nothing.
template <int TW, int TH, int TJ, bool kLooped = false>
__device__ inline void relax_blk(const Graph &s, int64_t lb, int mode, int max_rounds, int pass)
{
    constexpr int HW = TW + 2, HH = TH + 2, HJ = TJ + 2;
    constexpr int NH = HW * HH * HJ, NI = TW * TH * TJ;
    static_assert(NI % kBlock == 0 && NI / kBlock <= 32, "tile must hold 1..32 nodes per thread");
    constexpr int NPT = NI / kBlock;
    __shared__ int32_t sv[NH];
    __shared__ uint16_t smk[NI];
    // mode 0: BFS distance to the deficits in ht; mode 1: reachability in aux
    int32_t *__restrict__ val = mode == 0 ? s.ht : s.aux;
    const int step = mode == 0 ? 1 : 0;
    int32_t *flags = s.hdr->flags;
    int32_t *__restrict__ stamps = s.stamps;
    const int ntx = (s.W + TW - 1) / TW, nty = (s.H + TH - 1) / TH, ntz = (s.J + TJ - 1) / TJ;
    // In a loop over many tiles (kLooped) the thread index goes through an
    // empty asm statement: otherwise every per-thread offset of the tile is
    // hoisted out of the loop and stays live across it (87 registers instead
    // of 45 for an 8x8x16 tile).
    int tid = threadIdx.x;
    if (kLooped) asm volatile("" : "+v"(tid));
    if (pass > 1 && flags[(pass - 1) % kMaxFlags] == 0) return;     // converged already
    const int tile = (int)lb;
    const int bx = tile % ntx, by = (tile / ntx) % nty, bz = tile / (ntx * nty);
    // Thread t < 27 reads the stamp of tile t of the 3x3x3 neighbourhood (one
    // round trip instead of 27 in a row); neighbouring tiles may rewrite
    // their stamps during this pass, so the block-wide OR of what was read
    // decides for the whole block.
    // (a listed tile passed this test when the list was made)
    if (!kLooped) {
        int changed = pass == 1;
        if (pass > 1 && tid < 27) {
            const int tz = bz + tid / 9 - 1, ty = by + (tid / 3) % 3 - 1, tx = bx + tid % 3 - 1;
            if (tz >= 0 && tz < ntz && ty >= 0 && ty < nty && tx >= 0 && tx < ntx)
                changed = (stamps[(tz * nty + ty) * ntx + tx] >> 1) == pass - 1;
        }
        if (!__syncthreads_or(changed)) return;
    } else {
        __syncthreads();                     // the tile before may still read the shared arrays
    }
    const int x0 = bx * TW, y0 = by * TH, j0 = bz * TJ;

    // Halo values and masks: all of a thread's loads are issued before the
    // first wait; a position outside the grid reads element 0 (in bounds)
    // and is replaced by infinity / an empty mask.
    constexpr int NHT = (NH + kBlock - 1) / kBlock;
    int32_t hv[NHT];
    bool hin[NHT];
#pragma unroll
    for (int k = 0; k < NHT; ++k) {
        const int i = tid + k * kBlock;
        const int lx = i % HW, t = i / HW, ly = t % HH, lj = t / HH;
        const int gx = x0 + lx - 1, gy = y0 + ly - 1, gj = j0 + lj - 1;
        hin[k] = i < NH && gx >= 0 && gx < s.W && gy >= 0 && gy < s.H && gj >= 0 && gj < s.J;
        hv[k] = val[hin[k] ? ((int64_t)gj * s.H + gy) * s.W + gx : 0];
    }
    uint16_t mv[NPT];
    bool mok[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = tid + k * kBlock;
        const int lx = i % TW, t = i / TW, ly = t % TH, lj = t / TH;
        const int gx = x0 + lx, gy = y0 + ly, gj = j0 + lj;
        mok[k] = gx < s.W && gy < s.H && gj < s.J;
        mv[k] = s.mask[mok[k] ? ((int64_t)gj * s.H + gy) * s.W + gx : 0];
    }
#pragma unroll
    for (int k = 0; k < NHT; ++k) {
        const int i = tid + k * kBlock;
        if (i < NH) sv[i] = hin[k] ? hv[k] : kInf;
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) smk[tid + k * kBlock] = mok[k] ? mv[k] : (uint16_t)0;
    constexpr int hoff[14] = {
        (dir_dj(0) * HH + dir_dy(0)) * HW + dir_dx(0),   (dir_dj(1) * HH + dir_dy(1)) * HW + dir_dx(1),
        (dir_dj(2) * HH + dir_dy(2)) * HW + dir_dx(2),   (dir_dj(3) * HH + dir_dy(3)) * HW + dir_dx(3),
        (dir_dj(4) * HH + dir_dy(4)) * HW + dir_dx(4),   (dir_dj(5) * HH + dir_dy(5)) * HW + dir_dx(5),
        (dir_dj(6) * HH + dir_dy(6)) * HW + dir_dx(6),   (dir_dj(7) * HH + dir_dy(7)) * HW + dir_dx(7),
        (dir_dj(8) * HH + dir_dy(8)) * HW + dir_dx(8),   (dir_dj(9) * HH + dir_dy(9)) * HW + dir_dx(9),
        (dir_dj(10) * HH + dir_dy(10)) * HW + dir_dx(10), (dir_dj(11) * HH + dir_dy(11)) * HW + dir_dx(11),
        (dir_dj(12) * HH + dir_dy(12)) * HW + dir_dx(12), (dir_dj(13) * HH + dir_dy(13)) * HW + dir_dx(13)};
    __syncthreads();
    int32_t orig[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = tid + k * kBlock;
        const int lx = i % TW, t = i / TW, ly = t % TH, lj = t / TH;
        orig[k] = sv[((lj + 1) * HH + (ly + 1)) * HW + (lx + 1)];
    }

    // Within a round each thread takes its nodes in sequence and sees its own
    // updates at once, so it helps if they are consecutive levels of one
    // column, visited in the direction values travel: a round then carries a
    // value several levels along the chain instead of one.  Thread t owns
    // column t % C of the tile's C = TW * TH columns and NPT consecutive
    // levels (when the block covers the columns a whole number of times;
    // otherwise i = t + k * kBlock, which keeps a column's levels in one
    // thread when C is a multiple of kBlock).  Distances to the deficits
    // (mode 0) grow upwards from the bottom of the chain, reachability from
    // the excess (mode 1) spreads downwards; odd rounds take the reverse order.
    constexpr int C = TW * TH;
    constexpr bool kColumns = C <= kBlock && kBlock % C == 0;
    bool capped = true;
    for (int round = 0; round < max_rounds; ++round) {
        bool ch = false;
        const bool upward = ((round & 1) == 0) == (mode == 0);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int kk = upward ? NPT - 1 - k : k;
            const int i = kColumns ? tid % C + C * (NPT * (tid / C) + kk) : tid + kk * kBlock;
            const unsigned m = smk[i];
            if (!m) continue;
            const int lx = i % TW, t = i / TW, ly = t % TH, lj = t / TH;
            const int hi = ((lj + 1) * HH + (ly + 1)) * HW + (lx + 1);
            const int32_t c = sv[hi];
            int32_t best = c;
#pragma unroll
            for (int d = 0; d < 14; ++d)
                if ((m >> d) & 1u) {
                    const int32_t nv = sv[hi + hoff[d]] + step;
                    best = nv < best ? nv : best;
                }
            if (best < c) {
                sv[hi] = best;
                ch = true;
            }
        }
        if (!__syncthreads_or(ch)) { capped = false; break; }
    }
    bool wrote = false;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = tid + k * kBlock;
        const int lx = i % TW, t = i / TW, ly = t % TH, lj = t / TH;
        const int32_t v = sv[((lj + 1) * HH + (ly + 1)) * HW + (lx + 1)];
        if (v != orig[k]) {
            val[((int64_t)(j0 + lj) * s.H + (y0 + ly)) * s.W + (x0 + lx)] = v;
            wrote = true;
        }
    }
    const bool any_wrote = __syncthreads_or(wrote);
    if (tid == 0) {
        if (any_wrote || capped) {
            stamps[tile] = (pass << 1) | (capped ? 1 : 0);
            flags[pass % kMaxFlags] = 1;
        } else if (pass == 1) {
            stamps[tile] = 0;
        }
    }
}

// The relaxation pass of a compact thin skin: a tile holds 16 x 16 sites
// with all their stored levels (at most TJ), so every arc between two of its
// sites stays inside the tile whatever the windows' offsets; the LDS
// neighbour of a node across a site boundary is dj + wlo(own) - wlo(other)
// levels away.  Thread t owns the column of site t, whose levels it takes in
// the order values travel.  Change stamps, flags and rounds as relax_blk.
constexpr int kSkinTile = 16;

template <int TJ>
__global__ void __launch_bounds__(kBlock)
k_relax_skin(Graph s, int mode, int max_rounds, int pass)
{
    static_assert(kSkinTile * kSkinTile == kBlock, "one column per thread");
    constexpr int HW = kSkinTile + 2, HS = HW * HW, NH = HS * TJ;
    __shared__ int32_t sv[NH];
    __shared__ uint16_t smk[kBlock * TJ];
    __shared__ int32_t slo[HS];
    int32_t *__restrict__ val = mode == 0 ? s.ht : s.aux;
    const int step = mode == 0 ? 1 : 0;
    int32_t *flags = s.hdr->flags;
    int32_t *__restrict__ stamps = s.stamps;
    const int ntx = (s.W + kSkinTile - 1) / kSkinTile, nty = (s.H + kSkinTile - 1) / kSkinTile;
    const int tid = threadIdx.x;
    if (pass > 1 && flags[(pass - 1) % kMaxFlags] == 0) return;     // converged already
    const int tile = blockIdx.x;
    const int bx = tile % ntx, by = tile / ntx;
    int changed = pass == 1;
    if (pass > 1 && tid < 9) {
        const int ty = by + tid / 3 - 1, tx = bx + tid % 3 - 1;
        if (ty >= 0 && ty < nty && tx >= 0 && tx < ntx) changed = (stamps[ty * ntx + tx] >> 1) == pass - 1;
    }
    if (!__syncthreads_or(changed)) return;
    const int x0 = bx * kSkinTile, y0 = by * kSkinTile;

    constexpr int NHT = (NH + kBlock - 1) / kBlock;
    int32_t hv[NHT];
    bool hin[NHT];
#pragma unroll
    for (int k = 0; k < NHT; ++k) {
        const int i = tid + k * kBlock;
        const int lx = i % HW, ly = (i / HW) % HW, t = i / HS;
        const int gx = x0 + lx - 1, gy = y0 + ly - 1;
        hin[k] = i < NH && gx >= 0 && gx < s.W && gy >= 0 && gy < s.H && t < s.J;
        hv[k] = val[hin[k] ? (int64_t)t * s.plane + (int64_t)gy * s.W + gx : 0];
    }
    for (int i = tid; i < HS; i += kBlock) {
        const int gx = x0 + i % HW - 1, gy = y0 + i / HW - 1;
        slo[i] = (gx >= 0 && gx < s.W && gy >= 0 && gy < s.H) ? s.wlo[(int64_t)gy * s.W + gx] : 0;
    }
    const int cx = tid % kSkinTile, cy = tid / kSkinTile;       // this thread's site
    const int gx = x0 + cx, gy = y0 + cy;
    const bool site_in = gx < s.W && gy < s.H;
    uint16_t mv[TJ];
#pragma unroll
    for (int t = 0; t < TJ; ++t)
        mv[t] = s.mask[(site_in && t < s.J) ? (int64_t)t * s.plane + (int64_t)gy * s.W + gx : 0];
#pragma unroll
    for (int k = 0; k < NHT; ++k) {
        const int i = tid + k * kBlock;
        if (i < NH) sv[i] = hin[k] ? hv[k] : kInf;
    }
#pragma unroll
    for (int t = 0; t < TJ; ++t) smk[t * kBlock + tid] = (site_in && t < s.J) ? mv[t] : (uint16_t)0;
    __syncthreads();
    // LDS offsets of the 14 neighbours of this thread's nodes
    const int own = (cy + 1) * HW + (cx + 1);
    int off[14];
#pragma unroll
    for (int d = 0; d < 14; ++d) {
        const int other = own + dir_dy(d) * HW + dir_dx(d);
        off[d] = (dir_dj(d) + slo[own] - slo[other]) * HS + dir_dy(d) * HW + dir_dx(d);
    }
    int32_t orig[TJ];
#pragma unroll
    for (int t = 0; t < TJ; ++t) orig[t] = sv[t * HS + own];

    bool capped = true;
    for (int round = 0; round < max_rounds; ++round) {
        bool ch = false;
        const bool upward = ((round & 1) == 0) == (mode == 0);
#pragma unroll
        for (int k = 0; k < TJ; ++k) {
            const int t = upward ? TJ - 1 - k : k;
            const unsigned m = smk[t * kBlock + tid];
            if (!m) continue;
            const int hi = t * HS + own;
            const int32_t c = sv[hi];
            int32_t best = c;
#pragma unroll
            for (int d = 0; d < 14; ++d)
                if ((m >> d) & 1u) {
                    const int32_t nv = sv[hi + off[d]] + step;
                    best = nv < best ? nv : best;
                }
            if (best < c) {
                sv[hi] = best;
                ch = true;
            }
        }
        if (!__syncthreads_or(ch)) { capped = false; break; }
    }
    bool wrote = false;
#pragma unroll
    for (int t = 0; t < TJ; ++t) {
        const int32_t v = sv[t * HS + own];
        if (v != orig[t]) {
            val[(int64_t)t * s.plane + (int64_t)gy * s.W + gx] = v;
            wrote = true;
        }
    }
    const bool any_wrote = __syncthreads_or(wrote);
    if (tid == 0) {
        if (any_wrote || capped) {
            stamps[tile] = (pass << 1) | (capped ? 1 : 0);
            flags[pass % kMaxFlags] = 1;
        } else if (pass == 1) {
            stamps[tile] = 0;
        }
    }
}

template <int TW, int TH, int TJ, class Src>
__global__ void __launch_bounds__(kBlock)
k_relax(Src src, int mode, int max_rounds, int pass)
{
    constexpr bool kLooped = std::is_same<Src, Listed>::value;
    for_blocks(src, 1, [&](const Graph &s, int64_t lb) {
        relax_blk<TW, TH, TJ, kLooped>(s, lb, mode, max_rounds, pass);
    });
}

__device__ inline void count_blk(const Graph &s, int64_t lb)
{
    int64_t n = lb * kBlock + threadIdx.x;
    int a = 0, hmax = 0;
    if (n < s.N) {
        const int32_t h = s.ht[n];
        a = (s.ex[n] > 0 && h < kInf) ? 1 : 0;
        hmax = a ? h : 0;
    }
    const bool wave_active = wave_any(a != 0);
    if (lane0()) {                            // group flags of the sweeps that follow
        const int64_t g = group_of(lb);
        s.bact[g] = wave_active;
        s.binf[g] = 0;
    }
    a = block_sum(a);
    hmax = block_max(hmax);
    if (threadIdx.x == 0 && a) {
        atomicAdd(&my_slot(s.slots, lb).active, a);
        atomicMax(&my_slot(s.slots, lb).max_height, hmax);
    }
}

template <class Src>
__global__ void __launch_bounds__(kBlock)
k_count_active(Src src)
{
    for_blocks(src, 0, [&](const Graph &s, int64_t lb) { count_blk(s, lb); });
}

__global__ void k_zero_header(DevHeader *h, int what)
{
    int i = threadIdx.x;
    if (what == 0) {                 // everything
        if (i < kMaxFlags) h->flags[i] = 0;
        if (i == 0) { h->active = 0; h->prefix_err = 0; h->pushes = 0; h->visits = 0; }
        if (i < 4) h->lists[i] = 0;
    } else if (what == 1) {          // relaxation flags
        if (i < kMaxFlags) h->flags[i] = 0;
    } else if (what == 2) {          // active counter
        if (i == 0) h->active = 0;
    } else if (what == 3) {          // work-list lengths
        if (i < 4) h->lists[i] = 0;
    }
}

// Clears the change flags of passes first .. first+count-1.
__global__ void k_zero_flags(DevHeader *h, int first, int count)
{
    int i = threadIdx.x;
    if (i < count) h->flags[(first + i) % kMaxFlags] = 0;
}

// Clears the result and the read-out error bits; a data term outside
// [0, cap] seen by the build stays flagged until the graph is rebuilt.
__global__ void k_zero_result(int64_t *r, DevHeader *h)
{
    if (threadIdx.x == 0) { r[0] = 0; r[1] = 0; if (h) h->prefix_err &= kCostErr; }
}

// Labels: X = source-side nodes in the column, which must form the prefix
// v_1..v_X.  from_aux: a node is on the source side when the reachability
// relaxation reached it (aux == 0, minimal source side); otherwise when no
// deficit is reachable from it (infinite distance in ht, maximal source
// side).  In a thin-skin graph the levels at or above the window's top are
// source side by construction.
__global__ void __launch_bounds__(kBlock)
k_labels(Graph s, int32_t *__restrict__ labels, int from_aux)
{
    int64_t site = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (site >= s.plane) return;
    const int lo = s.win ? s.wlo[site] : 0, hi = s.win ? s.whi[site] : s.J;
    int X = lo;
    bool gap = false, bad = false;
    for (int j = lo; j < hi; ++j) {
        const int64_t n = (int64_t)(s.cw ? j - lo : j) * s.plane + site;
        bool in = from_aux ? s.aux[n] == 0 : s.ht[n] >= kInf;
        if (in) { if (gap) bad = true; ++X; }
        else gap = true;
    }
    labels[site] = X;
    if (bad) atomicOr(&s.hdr->prefix_err, 1);
}

__device__ inline long long pair_term(int h1, int h2, int d)
{
    int a = d < 0 ? -d : d;
    return (long long)h1 * a + (a > 1 ? (long long)h2 * (a - 1) : 0LL);
}

// E(X) from its definition (and the direct s -> t flow when m == 1).
__global__ void __launch_bounds__(kBlock)
k_energy(const int32_t *__restrict__ cost, const int32_t *__restrict__ labels, int W, int H,
         int m, int ph, int ih, int pv, int iv, Slot *__restrict__ slots)
{
    int64_t site = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    long long e = 0, tcap = 0;
    const int64_t plane = (int64_t)W * H;
    if (site < plane) {
        int y = (int)(site / W), x = (int)(site - (int64_t)y * W);
        int X = labels[site];
        e = cost[(int64_t)X * plane + site];
        if (x + 1 < W) e += pair_term(ph, ih, X - labels[site + 1]);
        if (y + 1 < H) e += pair_term(pv, iv, X - labels[site + W]);
        if (m == 1) tcap = cost[site];          // no nodes: every s -> t arc carries g(0)
    }
    e = block_sum(e);
    __syncthreads();
    tcap = block_sum(tcap);
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&my_slot(slots, blockIdx.x).e0, (unsigned long long)e);
        atomicAdd((unsigned long long *)&my_slot(slots, blockIdx.x).e1, (unsigned long long)tcap);
    }
}

// Deficits still unfilled (subtracted from the sink-side capacity).
__global__ void __launch_bounds__(kBlock)
k_deficit(Graph s)
{
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    long long d = 0;
    if (n < s.N) { int32_t e = s.ex[n]; d = e < 0 ? -(long long)e : 0; }
    d = block_sum(d);
    if (threadIdx.x == 0 && d)
        atomicAdd((unsigned long long *)&my_slot(s.slots, blockIdx.x).e1, (unsigned long long)(-d));
}

// Clears slot fields: what 0 = everything, 1 = active, 2 = energy/flow.
__global__ void __launch_bounds__(kSlots)
k_zero_slots(Slot *slots, int what)
{
    Slot &sl = slots[threadIdx.x];
    if (what == 0) {
        sl.pushes = 0; sl.visits = 0; sl.active = 0; sl.max_height = 0; sl.e0 = 0; sl.e1 = 0;
        sl.tcap = 0; sl.c0 = 0;
    }
    else if (what == 1) { sl.active = 0; sl.max_height = 0; }
    else { sl.e0 = 0; sl.e1 = 0; }
}

// Folds the slots: what 0 -> hdr->active, 1 -> hdr->pushes,
// 2 -> result[0] = energy, result[1] = flow (sink capacity + c0 - deficits),
// 3 -> hdr->tcap, hdr->c0 after a build, 4 -> hdr->seeded after a warm
// start, 5 -> 0 and 1 after a termination count, whose slots it then clears
// for the next count.
__global__ void __launch_bounds__(kSlots)
k_fold_slots(Slot *slots, DevHeader *hdr, int what, int64_t *result)
{
    static_assert(kSlots == kBlock, "one thread per slot");
    Slot &sl = slots[threadIdx.x];
    if (what == 5) {
        const int a0 = sl.active, m0 = sl.max_height;
        const int a = block_sum(a0);
        __syncthreads();
        const int m = block_max(m0);
        __syncthreads();
        const unsigned long long p = block_sum(sl.pushes);
        __syncthreads();
        const unsigned long long v = block_sum(sl.visits);
        if (threadIdx.x == 0) { hdr->active = a; hdr->max_height = m; hdr->pushes = p; hdr->visits = v; }
        sl.active = 0;                        // each thread clears the slot it read
        sl.max_height = 0;
    } else if (what == 0) {
        int a = block_sum(sl.active);
        __syncthreads();
        int m = block_max(sl.max_height);
        if (threadIdx.x == 0) { hdr->active = a; hdr->max_height = m; }
    } else if (what == 1) {
        unsigned long long p = block_sum(sl.pushes);
        __syncthreads();
        unsigned long long v = block_sum(sl.visits);
        if (threadIdx.x == 0) { hdr->pushes = p; hdr->visits = v; }
    } else if (what == 2) {
        long long e0 = block_sum(sl.e0);
        __syncthreads();
        long long e1 = block_sum(sl.e1);
        if (threadIdx.x == 0) { result[0] = e0; result[1] = e1 + hdr->tcap + hdr->c0; }
    } else if (what == 3) {
        long long t = block_sum(sl.tcap);
        __syncthreads();
        long long c = block_sum(sl.c0);
        if (threadIdx.x == 0) { hdr->tcap = t; hdr->c0 = c; }
    } else {
        long long e0 = block_sum(sl.e0);
        if (threadIdx.x == 0) hdr->seeded = e0;
    }
}

// ---------------------------------------------------------------------------
// Wave-front passes (Sec. 4.4 runs one before its push-relabel loop; the
// paper omits the details) and the level-2 approximation (Sec. 4.5).
// ---------------------------------------------------------------------------

// Column pass of the exact solve (GC_OPT_WAVE_FIRST): one pass along every column, from the source end
// towards the sink end over the free levels; each node hands the chain arc
// towards the sink as much of its excess (its own plus what the pass brought
// from below) as the arc's residual allows.  Heights are ignored, so a
// global relabel must follow before any push sweep.  One thread per site;
// the grid covers the sites with the node blocks of the source (a graph or a
// batch), blocks past the plane exit.
template <class Src>
__global__ void __launch_bounds__(kBlock)
k_wave(Src src)
{
    for_blocks(src, 0, [&](const Graph &s, int64_t lb) {
    if (lb * kBlock >= s.plane) return;             // whole block past the plane
    const int64_t site = lb * kBlock + threadIdx.x;
    int cnt = 0;
    if (site < s.plane) {
        const int lo = s.win ? s.wlo[site] : 0, hi = s.win ? s.whi[site] : s.J;
        int32_t carry = 0;
        for (int k = lo + 1; k <= hi; ++k) {
            const int64_t n = (int64_t)(s.cw ? k - 1 - lo : k - 1) * s.plane + site;
            const int32_t e0 = s.ex[n];
            int32_t e = e0 + carry;
            carry = 0;
            if (k < hi && e > 0) {
                const int32_t r = s.rd[n];
                const int32_t d = e < r ? e : r;
                if (d > 0) {
                    s.rd[n] = r - d;
                    e -= d;
                    carry = d;
                    ++cnt;
                }
            }
            if (e != e0) s.ex[n] = e;
        }
    }
    cnt = block_sum(cnt);
    if (threadIdx.x == 0 && cnt) atomicAdd(&my_slot(s.slots, lb).pushes, (unsigned long long)cnt);
    });
}

// Level 2, wave step (push half): every node with excess and a finite
// height pushes, arc by arc in direction order, min(excess, residual) to the
// neighbours exactly one below it.  Heights come from `hc` and are not
// written here, so along an arc pair at most one end is admissible and each
// pair word has one writer; inflow is summed into ein (integer atomics,
// order-free), so the step's result does not depend on the schedule.
// Forced levels of the skin have infinite height and are never admissible.
template <class T>
__global__ void __launch_bounds__(kBlock)
k_wave_push(Graph s, const int32_t *__restrict__ hc)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= s.N) return;
    int32_t e = s.ex[n];
    const int32_t h = hc[n];
    if (e <= 0 || h >= kInf) return;
    int j, y, x;
    decode(s, n, j, y, x);
    const T tp(s, n, j, y, x);
    const unsigned ex_mask = tp.ex;
    int32_t hv[14];
#pragma unroll
    for (int d = 0; d < 14; ++d) {
        const bool ok = (ex_mask >> d) & 1u;
        hv[d] = ok ? hc[tp.nb(s, n, d)] : kInf;
    }
#pragma unroll
    for (int d = 0; d < 14; ++d) {
        if (e <= 0 || hv[d] != h - 1) continue;
        const int32_t w = *tp.wp(s, n, d);
        const int32_t r = res_from_word(s, d, w);
        if (r <= 0) continue;
        const int32_t delta = e < r ? e : r;
        *tp.wp(s, n, d) = word_is_forward(d) ? w - delta : w + delta;
        atomicAdd(&s.ein[tp.nb(s, n, d)], delta);
        e -= delta;
    }
    s.ex[n] = e;
}

// Level 2, wave step (relabel half): merges the inflow, then lifts every node
// holding excess to one above its lowest residual neighbour when that is
// higher.  Neighbour heights are read from `hc` and the new ones written to
// `hn` (every node, so `hn` is the whole next height field): a Jacobi step.
template <class T>
__global__ void __launch_bounds__(kBlock)
k_wave_relabel(Graph s, const int32_t *__restrict__ hc, int32_t *__restrict__ hn)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= s.N) return;
    const int32_t in = s.ein[n];
    const int32_t e = s.ex[n] + in;
    int32_t h = hc[n];
    if (in != 0) {
        s.ex[n] = e;
        s.ein[n] = 0;
    }
    if (e > 0 && h < kInf) {
        int j, y, x;
        decode(s, n, j, y, x);
        const T tp(s, n, j, y, x);
        const unsigned ex_mask = tp.ex;
        int32_t w[14], hv[14];
#pragma unroll
        for (int d = 0; d < 14; ++d) {
            const bool ok = (ex_mask >> d) & 1u;
            w[d] = load_word(s, tp, n, d, ok);
            hv[d] = ok ? hc[tp.nb(s, n, d)] : kInf;
        }
        int32_t hmin = kInf;
#pragma unroll
        for (int d = 0; d < 14; ++d)
            if (((ex_mask >> d) & 1u) && res_from_word(s, d, w[d]) > 0)
                hmin = hv[d] < hmin ? hv[d] : hmin;
        const int32_t nh = hmin >= kInf ? kInf : hmin + 1;
        h = nh > h ? nh : h;
    }
    hn[n] = h;
}

// Opposite arc direction (the arc from the neighbour back).
__host__ __device__ constexpr int dir_opposite(int d)
{
    return d <= D_N ? (d ^ 1)
         : d == D_EM ? D_WP : d == D_WP ? D_EM : d == D_EP ? D_WM : d == D_WM ? D_EP
         : d == D_SM ? D_NP : d == D_NP ? D_SM : d == D_SP ? D_NM : D_SP;
}

constexpr int kCutLanes = 64;        // one wavefront per block: b^3 <= 64 nodes
constexpr int kCutMaxRounds = 4096;

// Level 2, the push-relabel loop of one block: the free nodes of the b x b
// sites of one delegate point whose level k lies in label group k / b, with
// only the arcs between them.  One lane per node, state in LDS.  Rounds:
// exact in-block distances to the block's deficits (1 at a deficit), stop
// when no node with excess has a finite one, else 2n synchronous steps of
// the wave rule (push along arcs to a neighbour exactly one below, merge the
// inflow, Jacobi relabel), n the block's node count.  The block's final
// excess and the pair words of its inner arcs are written back.
// Grid: (delegate x, delegate y, group offset 0..2 from the delegate label - 1).
template <class T>
__global__ void __launch_bounds__(kCutLanes)
k_block_cut(Graph s, const int32_t *__restrict__ coarse_labels, int b)
{
    __shared__ int32_t e[kCutLanes], hgt[kCutLanes], hnew[kCutLanes], ein[kCutLanes];
    __shared__ int32_t res[kCutLanes][14];
    __shared__ uint8_t member[kCutLanes];
    const int l = threadIdx.x;
    const int wc = (s.W + b - 1) / b;
    const int Sc = coarse_labels[(int64_t)blockIdx.y * wc + blockIdx.x];
    const int G = Sc - 1 + (int)blockIdx.z;                   // label group of the block
    if (G < 0) return;                                         // uniform: whole workgroup
    const int lx = l % b, ly = (l / b) % b, lk = l / (b * b);
    const int x = blockIdx.x * b + lx, y = blockIdx.y * b + ly, k = G * b + lk;
    bool mem = false;
    int64_t n = 0;
    if (lk < b && x < s.W && y < s.H && k >= 1 && k <= s.Jf) {
        const int64_t site = (int64_t)y * s.W + x;
        const int lo = s.wlo[site];
        mem = k > lo && k <= s.whi[site];
        n = (int64_t)(s.cw ? k - 1 - lo : k - 1) * s.plane + site;
    }
    member[l] = mem ? 1 : 0;
    __syncthreads();
    const int nb = __syncthreads_count(mem);
    if (nb == 0) return;
    auto lnb = [&](int d) -> int {
        const int nx = lx + dir_dx(d), ny = ly + dir_dy(d), nk = lk + dir_dj(d);
        if (nx < 0 || nx >= b || ny < 0 || ny >= b || nk < 0 || nk >= b) return -1;
        const int q = (nk * b + ny) * b + nx;
        return member[q] ? q : -1;
    };
    e[l] = 0; ein[l] = 0;
#pragma unroll
    for (int d = 0; d < 14; ++d) res[l][d] = 0;
    if (mem) {
        int j_, y_, x_;
        decode(s, n, j_, y_, x_);
        const T tp(s, n, j_, y_, x_);
        const unsigned ex_mask = tp.ex;
        e[l] = s.ex[n];
#pragma unroll
        for (int d = 0; d < 14; ++d)
            if (((ex_mask >> d) & 1u) && lnb(d) >= 0)
                res[l][d] = res_from_word(s, d, *tp.wp(s, n, d));
    }
    __syncthreads();
    int round = 0;
    for (;; ++round) {
        if (round >= kCutMaxRounds) {
            if (l == 0) atomicOr(&s.hdr->prefix_err, 2);
            break;
        }
        // exact in-block distances (synchronous relaxation to the fixpoint)
        hgt[l] = (mem && e[l] < 0) ? 1 : kInf;
        __syncthreads();
        for (;;) {
            int32_t best = hgt[l];
            if (mem && e[l] >= 0) {
#pragma unroll
                for (int d = 0; d < 14; ++d) {
                    const int q = lnb(d);
                    if (q >= 0 && res[l][d] > 0 && hgt[q] + 1 < best) best = hgt[q] + 1;
                }
            }
            __syncthreads();
            const bool ch = best < hgt[l];
            if (ch) hgt[l] = best;
            if (!__syncthreads_or(ch)) break;
        }
        if (!__syncthreads_or(mem && e[l] > 0 && hgt[l] < kInf)) break;
        for (int t = 0; t < 2 * nb; ++t) {
            // push: heights read only
            if (mem && e[l] > 0 && hgt[l] < kInf) {
                int32_t ev = e[l];
#pragma unroll
                for (int d = 0; d < 14; ++d) {
                    const int q = lnb(d);
                    if (ev <= 0 || q < 0 || hgt[q] != hgt[l] - 1) continue;
                    const int32_t r = res[l][d];
                    if (r <= 0) continue;
                    const int32_t dl = ev < r ? ev : r;
                    res[l][d] = r - dl;
                    atomicAdd(&res[q][dir_opposite(d)], dl);
                    atomicAdd(&ein[q], dl);
                    ev -= dl;
                }
                e[l] = ev;
            }
            __syncthreads();
            if (mem) {
                e[l] += ein[l];
                ein[l] = 0;
            }
            __syncthreads();
            // relabel: neighbours' heights of the step's start
            int32_t nh = hgt[l];
            if (mem && e[l] > 0 && hgt[l] < kInf) {
                int32_t hmin = kInf;
#pragma unroll
                for (int d = 0; d < 14; ++d) {
                    const int q = lnb(d);
                    if (q >= 0 && res[l][d] > 0 && hgt[q] < hmin) hmin = hgt[q];
                }
                const int32_t c = hmin >= kInf ? kInf : hmin + 1;
                nh = c > nh ? c : nh;
            }
            hnew[l] = nh;
            __syncthreads();
            hgt[l] = hnew[l];
            __syncthreads();
        }
    }
    if (mem) {
        s.ex[n] = e[l];
        int j_, y_, x_;
        decode(s, n, j_, y_, x_);
        const T tp(s, n, j_, y_, x_);
        const unsigned ex_mask = tp.ex;
#pragma unroll
        for (int d = 0; d < 14; ++d)
            if (word_is_forward(d) && ((ex_mask >> d) & 1u) && lnb(d) >= 0)
                *tp.wp(s, n, d) = res[l][d];
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Relaxation passes of a global relabel that does not end the solve, when
// the options leave them at 0.  The distances spread from the deficits a
// tile per pass; most of a relabel's passes carry them laterally over long
// distances to excess that is far from any deficit, which the sweeps that
// follow can hardly move anyway.  Measured on 450x375x64 and 640x480x64
// pairs (seeded sets of 3 and 6), a cap of 12-20 passes took 35-45 % off
// the solve (8: slower at 450x375x64); on seven sets of 16-, 24- and
// 31-level pairs 8 passes were about 10 % faster than 16 (4: outliers of
// 2-3x, 6: within 3 % of 8).
constexpr int kRelabelPassesDeep = 16;
constexpr int kRelabelPassesShallow = 8;

// Depth (levels of the full graph) from which a graph counts as deep for
// the relabel period, the relaxation's in-tile rounds and the early-stopped
// relabels' pass cap.
constexpr int kDeepLevels = 32;

// Sweeps between global relabels (the first period; later ones adapt below
// it), 24 below kDeepLevels levels and 32 from there on.  With relabels
// stopped early a shorter period pays: 32 against 64 was 10-20 % faster on
// 320x240x16 and 384x288x16 (grey, colour, penalties 1 and 2) and
// 640x480x64 pairs, within noise on 450x375x64; once shallow relabels
// stopped after 8 passes, 24 against 32 was 2-5 % faster on five sets of
// 16-level grey pairs and 12 % on colour pairs, even on 24 and 31 levels,
// and 6 % slower on 450x375x64 (20 and 16: slower again).
constexpr int kRelabelPeriodShallow = 24;
constexpr int kRelabelPeriodDeep = 32;

// Only a solve's first relabels may stop early.  Heights set by an early-
// stopped relabel need not be a valid labelling, so flow may circulate from
// one such relabel to the next; from this relabel on every relabel is exact,
// the standard algorithm, which ends.
constexpr int kCappedRelabels = 24;

struct Opts {
    int period, max_sweeps, tw, th, tj, local_iters, flags, relabel_passes;
};

Opts resolve(const gc_solve_opts *o)
{
    Opts r{0, 1 << 20, 8, 8, 16, 0, 0, 0};  // period 0: by depth (base_period)
    if (o) {
        if (o->relabel_period > 0) r.period = o->relabel_period;
        if (o->max_sweeps > 0) r.max_sweeps = o->max_sweeps;
        if (o->tile_w > 0) r.tw = o->tile_w;
        if (o->tile_h > 0) r.th = o->tile_h;
        if (o->tile_j > 0) r.tj = o->tile_j;
        if (o->local_iters > 0) r.local_iters = o->local_iters;
        r.flags = o->flags;
        r.relabel_passes = o->relabel_passes < 0 ? -1 : o->relabel_passes;
    }
    return r;
}

template <class Src>
using RelaxFn = void (*)(Src, int, int, int);

// Tile shapes compiled for the relaxation pass (x, y, depth layers).
#define GC_RELAX_SHAPES(X)                                                        \
    X(8, 8, 16) X(16, 8, 16) X(16, 16, 16) X(32, 8, 16) X(32, 4, 16) X(64, 4, 16) \
    X(16, 16, 8) X(32, 8, 8) X(32, 16, 8) X(64, 8, 8) X(16, 16, 4) X(32, 16, 4)   \
    X(32, 32, 4) X(64, 16, 4) X(8, 8, 32) X(16, 8, 32) X(16, 16, 32)

template <class Src>
RelaxFn<Src> relax_kernel(int tw, int th, int tj)
{
    if (tw < kMinTileW || th < kMinTileH || tj < kMinTileJ) return nullptr;
#define GC_RELAX_CASE(a, b, c) \
    if (tw == a && th == b && tj == c) return k_relax<a, b, c, Src>;
    GC_RELAX_SHAPES(GC_RELAX_CASE)
#undef GC_RELAX_CASE
    return nullptr;
}

// Kernels by topology: a compact thin skin takes the SkinTopo variants and
// its own relaxation tiles (16 x 16 sites with all their stored levels).
inline void (*mask_kernel(const Graph &s))(Graph, int)
{
    return s.cw ? k_mask<Graph, SkinTopo> : k_mask<Graph, FullTopo>;
}

inline RelaxFn<Graph> relax_skin_kernel(int levels)
{
    return levels <= 2 ? k_relax_skin<2> : levels <= 5 ? k_relax_skin<5> : levels <= 8 ? k_relax_skin<8>
         : levels <= 11 ? k_relax_skin<11> : levels <= kSkinMaxLevels ? k_relax_skin<kSkinMaxLevels> : nullptr;
}

int64_t relax_tiles(const Graph &s, const Opts &o)
{
    if (s.cw) return (int64_t)((s.W + kSkinTile - 1) / kSkinTile) * ((s.H + kSkinTile - 1) / kSkinTile);
    return (int64_t)((s.W + o.tw - 1) / o.tw) * ((s.H + o.th - 1) / o.th) * ((s.J + o.tj - 1) / o.tj);
}

// In-tile rounds of a relaxation pass when the options leave them at 0:
// 4 below kDeepLevels levels, 8 from there on and in compact skins.
// Measured with relabels stopped early: 4 rounds were 4-8 % faster than 8 on
// seven sets of 16-, 24- and 31-level pairs, and 8 were 1.5x faster than 4
// on 450x375x64.
__host__ __device__ inline int relax_rounds(int opt_rounds, const Graph &s)
{
    return opt_rounds > 0 ? opt_rounds : (s.J < kDeepLevels && !s.cw) ? 4 : 8;
}

// Pass cap of a relabel that does not end the solve (0: none) from the
// option (> 0: that many, < 0: none, 0: by the depth of the full problem,
// which a thin skin inherits: its windows hold few levels, but its lateral
// distances are those of the deep problem).
__host__ __device__ inline int relabel_cap(int opt_passes, const Graph &s)
{
    return opt_passes > 0 ? opt_passes : opt_passes < 0 ? 0
         : s.Jf < kDeepLevels ? kRelabelPassesShallow : kRelabelPassesDeep;
}

// Sweep kind: the split pair when the flags ask for it, else the fused
// kernel.  Measured on MI355X with early-stopped relabels: on 64-level
// graphs (450x375, 640x480) the fused sweep solves 10-20 % faster; on
// 384x288x16 it takes about 10 % more sweeps but half the launches and
// solves 3-4 % faster (mean over four seed sets of 16 pairs; 2.5 % slower on
// one set of 320x240x16 pairs); on the approximations' coarse graphs and
// skins of 64-level problems 2-6 % faster.
inline bool sweep_fused(const Opts &o)
{
    return !(o.flags & GC_OPT_SPLIT_SWEEP);
}

// Work-list launches (sweeps over the listed blocks, relaxation passes over
// the listed tiles, each on a fixed grid of kListGrid workgroups) on request.
// One workgroup per block of the whole graph costs the dispatch of every
// block even when few hold an active node (about 10 us per sweep at 450x375
// with 64 depth numbers), but it lets a block that receives flow during a
// sweep run in that same sweep, since it tests its flags when dispatched;
// a list fixed before the sweep leaves it for the next one.  Measured on
// single graphs the lists needed up to 30 % more sweeps and solved 4-25 %
// slower (384x288x16, 450x375x64, 640x480x64), so they are off by default.
constexpr unsigned kListGrid = 2048;

// Workgroups of `kernel` (kBlock threads) that the GPU holds at once.  A
// persistent grid larger than this leaves the surplus waiting until a
// resident workgroup has finished its whole share, which doubles the time
// of an evenly split launch.
// Looked up once per (kernel, device) and kept.
template <class K>
unsigned resident_grid(K kernel)
{
    struct Entry { const void *k; int dev; unsigned grid; };
    static std::mutex mu;
    static Entry cache[64];
    static int used = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kListGrid;
    const void *key = reinterpret_cast<const void *>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < used; ++i)
        if (cache[i].k == key && cache[i].dev == dev) return cache[i].grid;
    int cus = 0, per_cu = 0;
    unsigned grid = kListGrid;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) == hipSuccess &&
        cus > 0 && per_cu > 0)
        grid = (unsigned)(cus * per_cu);
    if (used < 64) cache[used++] = Entry{key, dev, grid};
    return grid;
}

inline bool use_lists(const Opts &o, int64_t)
{
    return (o.flags & GC_OPT_LISTS) != 0;
}

inline unsigned list_grid(int64_t items, unsigned resident)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, resident));
}

// Sweeps until the next global relabel.  The first period is the full
// relabel period: its sweeps also saturate arcs, which keeps the following
// BFS small (cutting it short was measured to cost more relaxation passes
// than it saved sweeps).  After that, an active node at height h is h - 1
// arcs from a deficit, so a period of twice the largest active height (at
// least kMinPeriod) gives the remaining excess room to arrive; on 384x288x16
// pairs this cut 20 % of the sweeps at the same number of global relabels.
constexpr int kMinPeriod = 16;

__host__ __device__ inline int base_period(int opt_period, const Graph &s)
{
    return opt_period > 0 ? opt_period : s.Jf < kDeepLevels ? kRelabelPeriodShallow : kRelabelPeriodDeep;
}

__host__ __device__ inline int period_for_round(int opt_period, int flags, const Graph &s, int round,
                                                int max_active_height)
{
    const int base = base_period(opt_period, s);
    if (round == 0 || (flags & GC_OPT_FIXED_PERIOD)) return base;
    const int q = 2 * max_active_height;
    const int lo = base < kMinPeriod ? base : kMinPeriod;
    return q < lo ? lo : q > base ? base : q;
}

// The optional wave-front pass runs once, before the first global relabel
// (heights are all zero then, so ignoring them loses nothing).
inline bool wave_in_round(const Opts &o, int round)
{
    return round == 0 && (o.flags & GC_OPT_WAVE_FIRST) != 0;
}

int check_opts(const Opts &o)
{
    if (!relax_kernel<Graph>(o.tw, o.th, o.tj)) return GC_E_ARG;
    return GC_OK;
}

// Optional per-launch device timing: a pair of events around each launch on
// the solve stream, summed per kernel class once the stream has drained.
// Per-thread HIP objects are released when the thread ends (the batched
// solve runs graphs on short-lived worker threads).
struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};
thread_local EventPool t_pool;
thread_local std::vector<hipEvent_t> &t_events = t_pool.ev;

// One launch in kTimeEvery of each class is timed (events on every launch
// slow the host enough to leave the GPU idle between short sweeps); the class
// total is the sampled mean times the launch count.  Which launches are
// timed follows a hash of the launch's number within its class, counted
// over all solves of the host thread: a fixed stride aliases with the sweep
// periods and relaxation batches, and a count restarted per solve samples
// the same positions of every solve (both biased the mean by 5-17 % against
// the profiler's per-dispatch times; this scheme by under 2 % for the sweeps).  A timed launch carries
// its start and stop events in its own dispatch (hipExtLaunchKernelGGL), so
// the interval is the kernel's execution, as a profiler reports it, not the
// kernel plus the queue's event packets.
constexpr int kTimeEvery = 16;
// Graphs of at least this many nodes run few, long launches: one in 4 is
// timed there (one in 16 left the mean of a 640x480x64 solve's ~800 sweeps
// 19 % off the profiler's).
constexpr int64_t kTimeDenseNodes = int64_t(1) << 22;
constexpr int kTimeEveryLarge = 4;

inline bool timed_launch(int klass, int k, int every)
{
    uint32_t h = (uint32_t)k * 0x9E3779B1u + (uint32_t)klass * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    return (h % (uint32_t)every) == 0;
}

thread_local uint32_t t_class_launches[GC_K_CLASSES];

struct HeaderRead;

struct Launcher {
    hipStream_t st;
    bool timing;
    std::vector<int> cls;
    int launched[GC_K_CLASSES] = {};
    HeaderRead *rb = nullptr;          // read-back landing buffer; null: the thread's pinned one
    int every = kTimeEvery;            // one launch in `every` of a class is timed

    hipEvent_t event(size_t i)
    {
        while (t_events.size() <= i) {
            hipEvent_t e = nullptr;
            // no system-scope fence when the event is recorded: a fenced stop
            // event writes back and invalidates the L2 at the end of the timed
            // dispatch, which lengthened it (and slowed the launches after it)
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
            t_events.push_back(e);
        }
        return t_events[i];
    }

    template <typename K, typename... Args>
    void run(int klass, K kernel, dim3 grid, Args... args)
    {
        hipEvent_t a = nullptr, b = nullptr;
        if (timing && (++launched[klass], timed_launch(klass, (int)t_class_launches[klass]++, every))) {
            a = event(2 * cls.size());
            b = event(2 * cls.size() + 1);
        }
        if (!a || !b) {
            hipLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, st, args...);
            return;
        }
        hipExtLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, st, a, b, 0, args...);
        cls.push_back(klass);
    }

    // Call after the stream has been synchronised.
    void collect(gc_solve_stats *out)
    {
        double ms_sum[GC_K_CLASSES] = {};
        int timed[GC_K_CLASSES] = {};
        for (size_t i = 0; i < cls.size(); ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, t_events[2 * i], t_events[2 * i + 1]) == hipSuccess) {
                ms_sum[cls[i]] += ms;
                timed[cls[i]]++;
            }
        }
        for (int c = 0; c < GC_K_CLASSES; ++c) {
            if (!timed[c]) continue;
            out->kernel_launches[c] += launched[c];
            out->kernel_ms[c] += ms_sum[c] / timed[c] * launched[c];
        }
        cls.clear();
        for (int &n : launched) n = 0;
    }
};

// The leading part of DevHeader the host reads back after a batch of
// relaxation passes: the pass flags, the active count and the push count.
struct HeaderRead {
    int32_t flags[kMaxFlags];
    int32_t active;
    int32_t prefix_err;
    int32_t max_height;
    int32_t pad[13];
    unsigned long long pushes;
    unsigned long long visits;
};
static_assert(sizeof(HeaderRead) == offsetof(DevHeader, tcap), "header prefix layout");

// Pinned landing buffer for the read-backs, one per host thread (a pageable
// destination would add a staging copy to every read-back).
struct PinnedHeader {
    HeaderRead *buf = nullptr;
    HeaderRead fallback;
    bool tried = false;
    ~PinnedHeader()
    {
        if (buf) (void)hipHostFree(buf);
    }
};

HeaderRead *header_buffer()
{
    thread_local PinnedHeader h;
    if (!h.tried) {
        h.tried = true;
        if (hipHostMalloc((void **)&h.buf, sizeof(HeaderRead), hipHostMallocDefault) != hipSuccess)
            h.buf = nullptr;
    }
    return h.buf ? h.buf : &h.fallback;
}

// Runs relaxation passes until a pass changes nothing.  Passes are issued in
// growing batches (4, 8, then 15: fewer than the flag ring holds, so a batch
// never clears the flag of the pass before it) with one read-back per batch;
// a pass that follows a pass without change returns at once, so over-issuing
// is cheap.  With `count_active` every batch is followed by the termination
// count of the sweeps (active nodes, block flags) and the push total, read
// back with the flags: the values of the batch that reached the fixpoint are
// the final ones, so the termination test costs no read-back of its own.
// Passes go out in batches with one read-back each; a pass after one that
// changed nothing returns at once, so a batch longer than needed costs a
// few microseconds per extra pass while a read-back idles the GPU for a
// host round trip.  The first batch is `first_batch` passes (the caller's
// estimate), later ones double up to kMaxFlags - 1.
int relax_to_fixpoint(const Graph &s, int mode, const Opts &o, Launcher &L, int *passes_out,
                      bool count_active = false, HeaderRead *out = nullptr, int first_batch = 4,
                      int cap = 0, bool *exact = nullptr, int *last_pass = nullptr)
{
    // cap > 0: stop after that many passes (*exact = false if the last one
    // still changed a value).  *last_pass, if given, holds the number of the
    // pass to continue from (0: a fresh relaxation) and receives the last one.
    if (exact) *exact = true;
    const int64_t tiles = relax_tiles(s, o);
    RelaxFn<Graph> fn = s.cw ? relax_skin_kernel(s.J) : relax_kernel<Graph>(o.tw, o.th, o.tj);
    RelaxFn<Listed> fnl = relax_kernel<Listed>(o.tw, o.th, o.tj);
    if (!fn || !fnl) return GC_E_ARG;
    const bool listed = use_lists(o, s.N) && !s.cw;
    if (listed) hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(64), 0, L.st, s.hdr, 3);
    if (tiles <= 0 && !count_active) return GC_OK;
    const int max_passes = 1 << 22;
    const unsigned grid = grid_for(s.N);
    HeaderRead *h = L.rb ? L.rb : header_buffer();
    const int first = last_pass ? *last_pass : 0;
    int passes = first;
    int batch = first_batch < 1 ? 1 : first_batch > kMaxFlags - 1 ? kMaxFlags - 1 : first_batch;
    if (cap > 0 && batch > cap) batch = cap;
    for (;;) {
        hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, L.st, s.hdr, passes + 1, batch);
        for (int b = 1; b <= batch && tiles > 0; ++b) {
            const int pass = passes + b;
            if (listed) {
                hipLaunchKernelGGL(k_list_tiles, dim3(grid_for(tiles)), dim3(kBlock), 0, L.st, s, pass,
                                   pass & 1, o.tw, o.th, o.tj);
                const Listed ls{s, s.tlist, &s.hdr->lists[2 + (pass & 1)]};
                L.run(GC_K_RELAX, fnl, dim3(list_grid(tiles, resident_grid(fnl))), ls, mode, relax_rounds(o.local_iters, s),
                      pass);
            } else {
                L.run(GC_K_RELAX, fn, dim3((unsigned)tiles), s, mode, relax_rounds(o.local_iters, s), pass);
            }
        }
        if (count_active) {
            // the count's slots are clear: the solve clears them before its
            // first count and every fold after a count clears them again
            L.run(GC_K_OTHER, k_count_active<Graph>, dim3(grid), s);
            hipLaunchKernelGGL(k_fold_slots, dim3(1), dim3(kSlots), 0, L.st, s.slots, s.hdr, 5, nullptr);
        }
        if (!hip_ok(hipGetLastError())) return GC_E_HIP;
        const size_t bytes = count_active ? sizeof(HeaderRead) : sizeof(h->flags);
        if (!hip_ok(hipMemcpyAsync(h, s.hdr, bytes, hipMemcpyDeviceToHost, L.st))) return GC_E_HIP;
        if (!hip_ok(hipStreamSynchronize(L.st))) return GC_E_HIP;
        bool done = tiles <= 0;
        for (int b = 1; b <= batch && !done; ++b) {
            ++passes;
            if (!h->flags[passes % kMaxFlags]) done = true;
        }
        if (done) break;
        if (cap > 0 && passes - first >= cap) {
            if (exact) *exact = false;
            break;
        }
        if (passes - first >= max_passes) return GC_E_NOT_CONVERGED;
        batch = batch * 2 > kMaxFlags - 1 ? kMaxFlags - 1 : batch * 2;
        if (cap > 0 && batch > cap - (passes - first)) batch = cap - (passes - first);
    }
    if (out) *out = *h;
    *passes_out += passes - first;
    if (last_pass) *last_pass = passes;
    return GC_OK;
}

// Captured sweep periods of single-graph solves, a few per host thread,
// keyed by the graph view (workspace addresses, shape, pair totals) and the
// sweep options; the least recently used capture is dropped first.
struct SweepCapture {
    Graph key;
    int period = 0;
    bool fused = false;
    bool listed = false;
    hipGraphExec_t exec = nullptr;
    unsigned long long used = 0;
    ~SweepCapture()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};
constexpr int kSweepCaptures = 8;

// One relabel period of sweeps.  listed: each sweep kernel runs over the
// blocks a compaction launch lists just before it (the list lengths restart
// at zero for the period, so a captured period replays correctly).
void launch_period(const Graph &s, int period, bool fused, bool listed, Launcher &L)
{
    const unsigned grid = grid_for(s.N);
    const unsigned cgrid = grid_for(grid);
    int par = 0;
    auto list = [&](int which) {
        L.run(GC_K_OTHER, k_list_blocks, dim3(cgrid), s, par, which);
        const Listed ls{s, s.blist, &s.hdr->lists[par]};
        par ^= 1;
        return ls;
    };
    if (listed) hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(64), 0, L.st, s.hdr, 3);
    for (int i = 0; i < period; ++i) {
        if (fused) {
            if (listed)
                L.run(GC_K_PUSH, k_sweep<Listed>, dim3(list_grid(grid, resident_grid(k_sweep<Listed>))), list(0));
            else L.run(GC_K_PUSH, s.cw ? k_sweep<Graph, SkinTopo> : k_sweep<Graph, FullTopo>, dim3(grid), s);
        } else if (listed) {
            L.run(GC_K_PUSH, k_push<Listed>, dim3(list_grid(grid, resident_grid(k_push<Listed>))), list(1));
            L.run(GC_K_RELABEL, k_relabel<Listed>, dim3(list_grid(grid, resident_grid(k_relabel<Listed>))),
                  list(0));
        } else {
            L.run(GC_K_PUSH, s.cw ? k_push<Graph, SkinTopo> : k_push<Graph, FullTopo>, dim3(grid), s);
            L.run(GC_K_RELABEL, s.cw ? k_relabel<Graph, SkinTopo> : k_relabel<Graph, FullTopo>, dim3(grid), s);
        }
    }
    if (fused) L.run(GC_K_OTHER, k_merge<Graph>, dim3(grid), s);
}

int replay_period(const Graph &s, int period, bool fused, bool listed, hipStream_t st)
{
    thread_local SweepCapture cache[kSweepCaptures];
    thread_local unsigned long long tick = 0;
    SweepCapture *hit = nullptr, *victim = &cache[0];
    for (SweepCapture &c : cache) {
        if (c.exec && c.period == period && c.fused == fused && c.listed == listed &&
            !memcmp(&c.key, &s, sizeof(Graph))) {
            hit = &c;
            break;
        }
        if (!c.exec || c.used < victim->used) victim = &c;
    }
    if (!hit) {
        if (victim->exec) (void)hipGraphExecDestroy(victim->exec);
        victim->exec = nullptr;
        hipGraph_t g = nullptr;
        if (!hip_ok(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal))) return GC_E_HIP;
        Launcher Lc{st, false, {}};
        launch_period(s, period, fused, listed, Lc);
        if (!hip_ok(hipStreamEndCapture(st, &g))) return GC_E_HIP;
        const bool ok = hip_ok(hipGraphInstantiate(&victim->exec, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        if (!ok) { victim->exec = nullptr; return GC_E_HIP; }
        victim->key = s;
        victim->period = period;
        victim->fused = fused;
        victim->listed = listed;
        hit = victim;
    }
    hit->used = ++tick;
    return hip_ok(hipGraphLaunch(hit->exec, st)) ? GC_OK : GC_E_HIP;
}

int read_i32(const int32_t *dev, int32_t *host, hipStream_t st)
{
    if (!hip_ok(hipMemcpyAsync(host, dev, sizeof(int32_t), hipMemcpyDeviceToHost, st))) return GC_E_HIP;
    if (!hip_ok(hipStreamSynchronize(st))) return GC_E_HIP;
    return GC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

GC_API const char *gc_status_str(int status)
{
    switch (status) {
    case GC_OK: return "ok";
    case GC_E_ARG: return "invalid argument";
    case GC_E_SHAPE: return "invalid shape";
    case GC_E_WORKSPACE: return "workspace too small or misaligned";
    case GC_E_CAP_OVERFLOW: return "capacities could overflow int32";
    case GC_E_NOT_CONVERGED: return "iteration cap reached before convergence";
    case GC_E_HIP: return "HIP runtime error";
    case GC_E_PREFIX: return "cut column is not a prefix";
    }
    return "unknown status";
}

GC_API int gc_last_hip_error(void) { return t_last_hip; }

GC_API int gc_problem_check(const gc_problem *p)
{
    if (!p) return GC_E_ARG;
    if (p->width < 0 || p->height < 0 || p->labels < 1) return GC_E_SHAPE;
    if (p->cap < 0 || p->penalty_h < 0 || p->inhibit_h < 0 || p->penalty_v < 0 || p->inhibit_v < 0)
        return GC_E_ARG;
    int64_t n = node_count(p);
    if (n >= (int64_t(1) << 29)) return GC_E_SHAPE;
    int64_t sites = (int64_t)p->width * p->height;
    int64_t big = p->cap;
    int64_t pairs[4] = {2 * (int64_t)p->penalty_h, 2 * (int64_t)p->penalty_v, p->inhibit_h, p->inhibit_v};
    for (int64_t v : pairs) big = v > big ? v : big;
    if (sites * (int64_t)p->cap + big >= (int64_t(1) << 30)) return GC_E_CAP_OVERFLOW;
    return GC_OK;
}

static size_t footprint(const gc_problem *p, int compact_block)
{
    if (gc_problem_check(p) != GC_OK) return 0;
    size_t n = (size_t)node_count(p, compact_block);
    const size_t sites = (size_t)p->width * p->height;
    return align256(sizeof(DevHeader)) + align256(kSlots * sizeof(Slot)) + 11 * align256(n * 4) +
           align256(n * 2) + 2 * align256(sites * 4) + 2 * align256(flag_bytes((int64_t)n)) +
           2 * align256(max_tiles(p, compact_block) * 4) + align256((n + kBlock - 1) / kBlock * 4);
}

GC_API size_t gc_graph_footprint_bytes(const gc_problem *p)
{
    return footprint(p, 0);
}

GC_API size_t gc_skin_footprint_bytes(const gc_problem *p, int32_t block)
{
    return block >= 1 ? footprint(p, block) : 0;
}

GC_API int stereo_cost_volume(const uint8_t *left, const uint8_t *right, const gc_problem *p,
                              int32_t *cost, void *stream)
{
    int rc = gc_problem_check(p);
    if (rc == GC_E_CAP_OVERFLOW) rc = GC_OK;     // the cost volume itself cannot overflow
    if (rc != GC_OK) return rc;
    if (!left || !right || !cost) return GC_E_ARG;
    if (p->width == 0 || p->height == 0) return GC_OK;
    if (p->height > 65535 || p->labels > 65535) return GC_E_SHAPE;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid(grid_for(p->width), (unsigned)p->height, (unsigned)p->labels);
    hipLaunchKernelGGL(k_cost_volume, grid, dim3(kBlock), 0, st, left, right, p->width,
                       p->height, p->labels, p->cap, cost);
    return hip_ok(hipGetLastError()) ? GC_OK : GC_E_HIP;
}

GC_API int stereo_cost_volume_rgb(const uint8_t *left, const uint8_t *right, const gc_problem *p,
                                  int32_t *cost, void *stream)
{
    int rc = gc_problem_check(p);
    if (rc == GC_E_CAP_OVERFLOW) rc = GC_OK;     // the cost volume itself cannot overflow
    if (rc != GC_OK) return rc;
    if (!left || !right || !cost) return GC_E_ARG;
    if (p->width == 0 || p->height == 0) return GC_OK;
    if (p->height > 65535 || p->labels > 65535) return GC_E_SHAPE;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid(grid_for(p->width), (unsigned)p->height, (unsigned)p->labels);
    hipLaunchKernelGGL(k_cost_volume_rgb, grid, dim3(kBlock), 0, st, left, right, p->width,
                       p->height, p->labels, p->cap, cost);
    return hip_ok(hipGetLastError()) ? GC_OK : GC_E_HIP;
}

static int build_common(const gc_problem *p, const int32_t *cost, void *ws, size_t ws_bytes,
                        gc_graph *g_out, int32_t block, bool compact = false)
{
    int rc = gc_problem_check(p);
    if (rc != GC_OK) return rc;
    if (!cost || !ws || !g_out) return GC_E_ARG;
    if (((uintptr_t)ws & 255) != 0 || ws_bytes < footprint(p, compact ? block : 0)) return GC_E_WORKSPACE;
    g_out->ws = ws;
    g_out->ws_bytes = ws_bytes;
    g_out->p = *p;
    g_out->window_block = block;
    g_out->compact = compact ? 1 : 0;
    return GC_OK;
}

GC_API int graph_build(const gc_problem *p, const int32_t *cost, void *ws, size_t ws_bytes,
                       gc_graph *g_out, void *stream)
{
    int rc = build_common(p, cost, ws, ws_bytes, g_out, 0);
    if (rc != GC_OK) return rc;
    Graph s = view(g_out);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(64), 0, st, s.hdr, 0);
    hipLaunchKernelGGL(k_zero_slots, dim3(1), dim3(kSlots), 0, st, s.slots, 0);
    if (s.N > 0)
        hipLaunchKernelGGL(k_build<false>, dim3(grid_for(s.N)), dim3(kBlock), 0, st, s, cost,
                           p->labels, p->cap);
    hipLaunchKernelGGL(k_fold_slots, dim3(1), dim3(kSlots), 0, st, s.slots, s.hdr, 3, nullptr);
    return hip_ok(hipGetLastError()) ? GC_OK : GC_E_HIP;
}

GC_API int gc_coarse_problem(const gc_problem *p, int32_t block, gc_problem *coarse)
{
    if (!p || !coarse || block < 1) return GC_E_ARG;
    int rc = gc_problem_check(p);
    if (rc != GC_OK) return rc;
    const int64_t b = block, b2 = b * b;
    if (b2 * p->cap > INT32_MAX || b2 * p->penalty_h > INT32_MAX || b2 * p->penalty_v > INT32_MAX)
        return GC_E_CAP_OVERFLOW;
    gc_problem c;
    c.width = (int32_t)((p->width + b - 1) / b);
    c.height = (int32_t)((p->height + b - 1) / b);
    c.labels = (int32_t)((p->labels + b - 1) / b);
    c.cap = (int32_t)(b2 * p->cap);
    c.penalty_h = (int32_t)(b2 * p->penalty_h);
    c.penalty_v = (int32_t)(b2 * p->penalty_v);
    c.inhibit_h = p->inhibit_h;
    c.inhibit_v = p->inhibit_v;
    if ((rc = gc_problem_check(&c)) != GC_OK) return rc;
    *coarse = c;
    return GC_OK;
}

GC_API int coarse_cost_volume(const gc_problem *p, const int32_t *cost, int32_t block,
                              int32_t *coarse_cost, void *stream)
{
    gc_problem c;
    int rc = gc_coarse_problem(p, block, &c);
    if (rc != GC_OK) return rc;
    if (!cost || !coarse_cost) return GC_E_ARG;
    if (c.width == 0 || c.height == 0) return GC_OK;
    if (c.height > 65535 || c.labels > 65535) return GC_E_SHAPE;
    dim3 grid(grid_for(c.width), (unsigned)c.height, (unsigned)c.labels);
    hipLaunchKernelGGL(k_coarse_cost, grid, dim3(kBlock), 0, (hipStream_t)stream, cost, p->width,
                       p->height, p->labels, block, coarse_cost);
    return hip_ok(hipGetLastError()) ? GC_OK : GC_E_HIP;
}

GC_API int graph_build_window(const gc_problem *p, const int32_t *cost,
                              const int32_t *coarse_labels, int32_t block, void *ws,
                              size_t ws_bytes, gc_graph *g_out, void *stream)
{
    if (block < 1 || !coarse_labels) return GC_E_ARG;
    gc_problem c;
    int rc = gc_coarse_problem(p, block, &c);
    if (rc != GC_OK) return rc;
    if ((rc = build_common(p, cost, ws, ws_bytes, g_out, block)) != GC_OK) return rc;
    Graph s = view(g_out);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(64), 0, st, s.hdr, 0);
    hipLaunchKernelGGL(k_zero_slots, dim3(1), dim3(kSlots), 0, st, s.slots, 0);
    if (s.plane > 0)
        hipLaunchKernelGGL(k_windows, dim3(grid_for(s.plane)), dim3(kBlock), 0, st, s, coarse_labels,
                           block, p->labels);
    if (s.N > 0)
        hipLaunchKernelGGL(k_build<true>, dim3(grid_for(s.N)), dim3(kBlock), 0, st, s, cost,
                           p->labels, p->cap);
    hipLaunchKernelGGL(k_fold_slots, dim3(1), dim3(kSlots), 0, st, s.slots, s.hdr, 3, nullptr);
    return hip_ok(hipGetLastError()) ? GC_OK : GC_E_HIP;
}

GC_API int graph_build_skin(const gc_problem *p, const int32_t *cost, const int32_t *coarse_labels,
                            int32_t block, void *ws, size_t ws_bytes, gc_graph *g_out, void *stream)
{
    if (block < 1 || !coarse_labels) return GC_E_ARG;
    gc_problem c;
    int rc = gc_coarse_problem(p, block, &c);
    if (rc != GC_OK) return rc;
    if (stored_levels(p, block) > kSkinMaxLevels) return GC_E_ARG;
    if ((rc = build_common(p, cost, ws, ws_bytes, g_out, block, true)) != GC_OK) return rc;
    Graph s = view(g_out);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(64), 0, st, s.hdr, 0);
    hipLaunchKernelGGL(k_zero_slots, dim3(1), dim3(kSlots), 0, st, s.slots, 0);
    if (s.plane > 0) {
        hipLaunchKernelGGL(k_windows, dim3(grid_for(s.plane)), dim3(kBlock), 0, st, s, coarse_labels,
                           block, p->labels);
        hipLaunchKernelGGL(k_skin_c0, dim3(grid_for(s.plane)), dim3(kBlock), 0, st, s, p->labels);
    }
    if (s.N > 0)
        hipLaunchKernelGGL(k_build_skin, dim3(grid_for(s.N)), dim3(kBlock), 0, st, s, cost, p->labels,
                           p->cap);
    hipLaunchKernelGGL(k_fold_slots, dim3(1), dim3(kSlots), 0, st, s.slots, s.hdr, 3, nullptr);
    return hip_ok(hipGetLastError()) ? GC_OK : GC_E_HIP;
}

static int graph_check(const gc_graph *g)
{
    if (!g || !g->ws || g->window_block < 0) return GC_E_ARG;
    if (g->compact != 0 && (g->compact != 1 || g->window_block < 1)) return GC_E_ARG;
    int rc = gc_problem_check(&g->p);
    if (rc != GC_OK) return rc;
    if (g->compact && stored_levels(&g->p, g->window_block) > kSkinMaxLevels) return GC_E_ARG;
    if (g->ws_bytes < footprint(&g->p, g->compact ? g->window_block : 0)) return GC_E_WORKSPACE;
    return GC_OK;
}

// The exact solve of maxflow_solve.  rb: read-back landing buffer (null: the
// calling thread's pinned one).
static int solve_graph(gc_graph *g, const Opts &opt, gc_solve_stats *stats, hipStream_t st,
                       HeaderRead *rb)
{
    int rc;
    gc_solve_stats st_local;
    memset(&st_local, 0, sizeof(st_local));
    Graph s = view(g);
    if (s.N == 0) {
        if (stats) *stats = st_local;
        return GC_OK;
    }
    Launcher L{st, (opt.flags & GC_OPT_TIME_KERNELS) != 0, {}};
    if (s.N >= kTimeDenseNodes) L.every = kTimeEveryLarge;
    L.rb = rb;
    const unsigned grid = grid_for(s.N);
    const bool fused = sweep_fused(opt);
    const bool listed = use_lists(opt, s.N) && !s.cw;
    const bool use_graph = st != nullptr && (opt.flags & GC_OPT_SWEEP_GRAPH) != 0 && !L.timing;
    int status = GC_OK;
    int batch_hint = 4;
    hipLaunchKernelGGL(k_zero_slots, dim3(1), dim3(kSlots), 0, st, s.slots, 1);   // the counts' slots
    for (int round = 0;; ++round) {
        // wave-front pass along the columns, then exact global relabelling:
        // BFS distance to the deficit nodes
        if (wave_in_round(opt, round))
            L.run(GC_K_OTHER, k_wave<Graph>, dim3(grid_for(s.plane)), s);
        L.run(GC_K_OTHER, mask_kernel(s), dim3(grid), s, 0);
        L.run(GC_K_OTHER, k_seed<Graph>, dim3(grid), s, 0);
        if (!hip_ok(hipGetLastError())) return GC_E_HIP;
        // termination count and push total come back with the last flags;
        // the first batch of passes is sized from the previous relabel's
        HeaderRead hr;
        const int passes_before = st_local.bfs_passes;
        // a relabel may stop early (opt.relabel_passes); one that finds no
        // active node is carried on to its exact fixpoint, which alone ends
        // the solve
        bool exact = true;
        int last = 0;
        if ((rc = relax_to_fixpoint(s, 0, opt, L, &st_local.bfs_passes, true, &hr, batch_hint,
                                    round < kCappedRelabels ? relabel_cap(opt.relabel_passes, s) : 0, &exact,
                                    &last)) != GC_OK)
            return rc;
        if (hr.prefix_err & kCostErr) return GC_E_CAP_OVERFLOW;
        if (hr.active == 0 && !exact &&
            (rc = relax_to_fixpoint(s, 0, opt, L, &st_local.bfs_passes, true, &hr, batch_hint, 0, nullptr,
                                    &last)) != GC_OK)
            return rc;
        batch_hint = st_local.bfs_passes - passes_before + 1;
        st_local.global_relabels++;
        st_local.active_last = hr.active;
        st_local.pushes = (int64_t)hr.pushes;
        st_local.active_visits = (int64_t)hr.visits;
        if (hr.active == 0) break;
        const int period = period_for_round(opt.period, opt.flags, s, round, hr.max_height);
        if (st_local.sweeps >= opt.max_sweeps) { status = GC_E_NOT_CONVERGED; break; }
        if (use_graph) {
            if ((rc = replay_period(s, period, fused, listed, st)) != GC_OK) return rc;
        } else {
            launch_period(s, period, fused, listed, L);
        }
        st_local.sweeps += period;
        if (!hip_ok(hipGetLastError())) return GC_E_HIP;
    }
    // the last read-back synchronised the stream
    L.collect(&st_local);
    if (stats) *stats = st_local;
    return status;
}

GC_API int maxflow_solve(gc_graph *g, const gc_solve_opts *o, gc_solve_stats *stats, void *stream)
{
    int rc = graph_check(g);
    if (rc != GC_OK) return rc;
    Opts opt = resolve(o);
    if ((rc = check_opts(opt)) != GC_OK) return rc;
    return solve_graph(g, opt, stats, (hipStream_t)stream, nullptr);
}

__global__ void __launch_bounds__(kBlock)
k_zero_i32(int32_t *p, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_set_i64(int64_t *p, long long v)
{
    if (threadIdx.x == 0) *p = v;
}

// Warm start of an exact solve from a solved thin-skin graph of the same
// problem and data term.  The skin's build folded every arc between a free
// and a forced node: arcs from forced-source nodes were taken as saturated
// (their capacity added to the free node's excess), arcs into forced-sink
// nodes likewise (their capacity a deficit of the free node), and its stored
// words already hold those saturations.  The same flows on the full graph
// give a pseudoflow (capacities respected, imbalance anywhere): free nodes
// take the skin's excess and the words of their arcs, forced nodes keep the
// fresh build's words towards forced partners and get the imbalance of the
// saturated arcs (a forced-source node loses what it sent into the skin, a
// forced-sink node gains what it received).  Heights restart at 0: the
// solve begins with an exact global relabel.  Slots' e0 collects the total
// positive excess, which bounds every node's excess from then on.
template <bool kCompact>
__global__ void __launch_bounds__(kBlock)
k_warm_start(Graph f, Graph k, const int32_t *__restrict__ cost)
{
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    long long pos = 0;
    if (n < f.N) {
        int j, y, x;
        decode(f, n, j, y, x);
        const int64_t site = (int64_t)y * f.W + x;
        const int kk = j + 1;
        const int lo = k.wlo[site];
        const int cn = node_class(kk, lo, k.whi[site]);
        // the skin's copy of this node (a compact skin stores free levels only)
        const int64_t nk = kCompact ? (int64_t)(j - lo) * k.plane + site : n;
        const unsigned ex_mask = arc_exists(f, j, y, x);
        const int ph = f.te / 2, pv = f.ts / 2;
        int32_t e = 0;
#pragma unroll
        for (int d = 0; d < 14; ++d) {
            if (!((ex_mask >> d) & 1u)) continue;
            const int64_t psite = site + dir_dy(d) * (int64_t)f.W + dir_dx(d);
            const int cp = node_class(kk + dir_dj(d), k.wlo[psite], k.whi[psite]);
            int32_t cout = 0, cin = 0;
            if (cn != FREE && cp == FREE) arc_caps(f, cost, d, site, j, ph, pv, cout, cin);
            if (word_is_forward(d) && (cn == FREE || cp == FREE)) {
                // a forced node's word towards a free one never changes in the
                // skin (nothing is pushed into a forced node): its build value
                *word_ptr(f, n, d) = cn == FREE ? word_array(k, d)[nk]
                                   : !kCompact ? *word_ptr(k, n, d) : cn == FSNK ? cout + cin : 0;
            }
            if (cn != FREE && cp == FREE) e += cn == FSRC ? -cout : cin;
        }
        const int32_t ex = cn == FREE ? k.ex[nk] : f.ex[n] + e;
        f.ex[n] = ex;
        f.ht[n] = 0;
        f.ein[n] = 0;
        pos = ex > 0 ? ex : 0;
    }
    pos = block_sum(pos);
    if (threadIdx.x == 0 && pos) atomicAdd((unsigned long long *)&my_slot(f.slots, blockIdx.x).e0,
                                           (unsigned long long)pos);
}

GC_API int graph_warm_start(gc_graph *g, const gc_graph *skin, const int32_t *cost, void *stream)
{
    int rc = graph_check(g);
    if (rc != GC_OK) return rc;
    if ((rc = graph_check(skin)) != GC_OK) return rc;
    if (!cost || g->window_block != 0 || skin->window_block < 1) return GC_E_ARG;
    if (memcmp(&g->p, &skin->p, sizeof(gc_problem)) != 0) return GC_E_ARG;
    Graph f = view(g), k = view(skin);
    hipStream_t st = (hipStream_t)stream;
    if (f.N == 0) return GC_OK;
    hipLaunchKernelGGL(k_zero_slots, dim3(1), dim3(kSlots), 0, st, f.slots, 2);
    if (k.cw) hipLaunchKernelGGL(k_warm_start<true>, dim3(grid_for(f.N)), dim3(kBlock), 0, st, f, k, cost);
    else hipLaunchKernelGGL(k_warm_start<false>, dim3(grid_for(f.N)), dim3(kBlock), 0, st, f, k, cost);
    hipLaunchKernelGGL(k_fold_slots, dim3(1), dim3(kSlots), 0, st, f.slots, f.hdr, 4, nullptr);
    // the relaxation flags and activity flags of the fresh build stay valid:
    // the solve's first global relabel recomputes every height, and every
    // 64-node group is marked by its first termination count
    if (!hip_ok(hipGetLastError())) return GC_E_HIP;
    long long seeded = 0;
    if (!hip_ok(hipMemcpyAsync(&seeded, &f.hdr->seeded, sizeof(seeded), hipMemcpyDeviceToHost, st)))
        return GC_E_HIP;
    if (!hip_ok(hipStreamSynchronize(st))) return GC_E_HIP;
    // a node's excess never exceeds the total positive excess: keep it in int32
    return seeded >= (1LL << 30) ? GC_E_CAP_OVERFLOW : GC_OK;
}

GC_API int approx_level2_cut(gc_graph *skin, const int32_t *cost, const int32_t *coarse_labels,
                             int32_t wave_steps, int32_t *labels, int64_t *result, void *stream)
{
    int rc = graph_check(skin);
    if (rc != GC_OK) return rc;
    if (!cost || !coarse_labels || !labels || !result || wave_steps < 0) return GC_E_ARG;
    const int b = skin->window_block;
    if (b < 1 || b * b * b > kCutLanes) return GC_E_ARG;
    Graph s = view(skin);
    hipStream_t st = (hipStream_t)stream;
    const gc_problem &p = skin->p;
    Opts opt = resolve(nullptr);
    Launcher L{st, false, {}};
    int passes = 0;
    hipLaunchKernelGGL(k_zero_result, dim3(1), dim3(64), 0, st, result, s.hdr);
    if (s.N > 0) {
        const unsigned grid = grid_for(s.N);
        // initialisation: exact residual distances to the deficits
        hipLaunchKernelGGL(mask_kernel(s), dim3(grid), dim3(kBlock), 0, st, s, 0);
        hipLaunchKernelGGL(k_seed<Graph>, dim3(grid), dim3(kBlock), 0, st, s, 0);
        if (!hip_ok(hipGetLastError())) return GC_E_HIP;
        if ((rc = relax_to_fixpoint(s, 0, opt, L, &passes)) != GC_OK) return rc;
        // wave steps over the whole skin; heights alternate between ht and aux
        hipLaunchKernelGGL(k_zero_i32, dim3(grid), dim3(kBlock), 0, st, s.ein, s.N);
        int32_t *hc = s.ht, *hn = s.aux;
        for (int t = 0; t < wave_steps; ++t) {
            if (s.cw) {
                hipLaunchKernelGGL(k_wave_push<SkinTopo>, dim3(grid), dim3(kBlock), 0, st, s, hc);
                hipLaunchKernelGGL(k_wave_relabel<SkinTopo>, dim3(grid), dim3(kBlock), 0, st, s, hc, hn);
            } else {
                hipLaunchKernelGGL(k_wave_push<FullTopo>, dim3(grid), dim3(kBlock), 0, st, s, hc);
                hipLaunchKernelGGL(k_wave_relabel<FullTopo>, dim3(grid), dim3(kBlock), 0, st, s, hc, hn);
            }
            std::swap(hc, hn);
        }
        // every block's push-relabel loop on its own
        const dim3 bgrid((unsigned)((s.W + b - 1) / b), (unsigned)((s.H + b - 1) / b), 3);
        if (s.cw) hipLaunchKernelGGL(k_block_cut<SkinTopo>, bgrid, dim3(kCutLanes), 0, st, s, coarse_labels, b);
        else hipLaunchKernelGGL(k_block_cut<FullTopo>, bgrid, dim3(kCutLanes), 0, st, s, coarse_labels, b);
        // read-out: distances to the unfilled deficits; unreachable = source side
        hipLaunchKernelGGL(mask_kernel(s), dim3(grid), dim3(kBlock), 0, st, s, 0);
        hipLaunchKernelGGL(k_seed<Graph>, dim3(grid), dim3(kBlock), 0, st, s, 0);
        if (!hip_ok(hipGetLastError())) return GC_E_HIP;
        if ((rc = relax_to_fixpoint(s, 0, opt, L, &passes)) != GC_OK) return rc;
    }
    hipLaunchKernelGGL(k_zero_slots, dim3(1), dim3(kSlots), 0, st, s.slots, 2);
    if (s.plane > 0) {
        hipLaunchKernelGGL(k_labels, dim3(grid_for(s.plane)), dim3(kBlock), 0, st, s, labels, 0);
        hipLaunchKernelGGL(k_energy, dim3(grid_for(s.plane)), dim3(kBlock), 0, st, cost, labels,
                           p.width, p.height, p.labels, p.penalty_h, p.inhibit_h, p.penalty_v,
                           p.inhibit_v, s.slots);
    }
    hipLaunchKernelGGL(k_fold_slots, dim3(1), dim3(kSlots), 0, st, s.slots, s.hdr, 2, result);
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, st, result + 1, -1LL);
    if (!hip_ok(hipGetLastError())) return GC_E_HIP;
    int32_t perr = 0;
    if ((rc = read_i32(&s.hdr->prefix_err, &perr, st)) != GC_OK) return rc;
    return (perr & kCostErr) ? GC_E_CAP_OVERFLOW : (perr & 2) ? GC_E_NOT_CONVERGED
         : (perr & 1) ? GC_E_PREFIX : GC_OK;
}

// ---------------------------------------------------------------------------
// Batched solve: every member advances on the device.
//
// A batch is a device table of member graphs, each with a MemberCtl record
// of where its solve stands.  One step moves every member by one phase of
// the single-graph solve (the mask and seeds of a global relabel, one
// relaxation pass, the termination count, one push / relabel / fused sweep,
// the inflow merge), all members in the same launches:
//   k_batch_phase   one workgroup per member: reads what its last step left
//                   (a relaxation pass's change flag, the folded count) and
//                   picks the member's next phase, as maxflow_solve's host
//                   loop does;
//   k_batch_list    per member, the work list of the step (active blocks of
//                   a sweep, changed tiles of a relaxation pass);
//   k_batch_scan    prefix offsets of the members' work units;
//   k_batch_full, k_batch_relax, k_batch_sweeps
//                   each a fixed grid of workgroups that takes the units of
//                   one kind (every block; listed tiles; listed blocks) of all
//                   members in turn (the tile work queue) and runs the same
//                   device functions as the single-graph kernels.
// The host replays a captured sequence of steps and reads the members'
// records once per replay; nothing in a step waits for the host.
// ---------------------------------------------------------------------------

namespace {


__global__ void __launch_bounds__(kSlots)
k_batch_phase(BatchDev *T)
{
    const int g = blockIdx.x;
    MemberCtl &c = T->ctl[g];
    const Graph s = T->graphs[g];
    const int t = threadIdx.x;
    __shared__ int next;
    const int last = c.phase;
    __syncthreads();                         // every wave has read it before it changes
    if (last == BP_COUNT) {                  // fold the termination count
        const Slot &sl = s.slots[t];
        const int a = block_sum(sl.active);
        const int mh = block_max(sl.max_height);
        __syncthreads();
        const unsigned long long pu = block_sum(sl.pushes);
        __syncthreads();
        const unsigned long long vi = block_sum(sl.visits);
        if (t == 0) {
            c.active = a;
            c.max_height = mh;
            c.pushes = (long long)pu;
            c.visits = (long long)vi;
            c.relabels++;
        }
    }
    if (t == 0) {
        int nx = BP_DONE;
        switch (last) {
        case BP_INIT:
            nx = BP_SEED;
            break;
        case BP_SEED:
            nx = BP_RELAX;
            c.pass = 1;
            c.cut = 0;
            s.hdr->flags[1 % kMaxFlags] = 0;
            break;
        case BP_RELAX:
            c.passes++;
            if (!s.hdr->flags[c.pass % kMaxFlags]) {
                nx = BP_COUNT;                   // converged: exact
                c.cut = 0;
            } else if (c.cut != 2 && c.round < kCappedRelabels && relabel_cap(T->relabel_passes, s) > 0 &&
                       c.pass >= relabel_cap(T->relabel_passes, s)) {
                nx = BP_COUNT;                   // stopped early (as maxflow_solve)
                c.cut = 1;
            } else {
                nx = BP_RELAX;
                c.pass++;
                s.hdr->flags[c.pass % kMaxFlags] = 0;
            }
            break;
        case BP_COUNT:
            if (c.active == 0 && c.cut == 1) {  // carry the relabel on to its fixpoint
                nx = BP_RELAX;
                c.cut = 2;
                c.relabels--;                    // (one relabel, counted when it ends)
                c.pass++;
                s.hdr->flags[c.pass % kMaxFlags] = 0;
            } else if (c.active == 0 || c.sweeps >= T->max_sweeps) {
                nx = BP_DONE;
                c.status = c.active == 0 ? GC_OK : GC_E_NOT_CONVERGED;
                c.done_step = T->step;
            } else {
                c.period = period_for_round(T->period, T->flags, s, c.round, c.max_height);
                c.sweep = 0;
                nx = c.fused ? BP_SWEEP : BP_PUSH;
            }
            break;
        case BP_PUSH:
            nx = BP_RELABEL;
            break;
        case BP_RELABEL:
            c.sweep++;
            c.sweeps++;
            if (c.sweep >= c.period) { c.round++; nx = BP_SEED; }
            else nx = BP_PUSH;
            break;
        case BP_SWEEP:
            c.sweep++;
            c.sweeps++;
            nx = c.sweep >= c.period ? BP_MERGE : BP_SWEEP;
            break;
        case BP_MERGE:
            c.round++;
            nx = BP_SEED;
            break;
        default:
            nx = BP_DONE;
        }
        c.phase = nx;
        s.hdr->lists[0] = 0;                // the step's lists count from zero
        s.hdr->lists[2] = 0;
        next = nx;
    }
    __syncthreads();
    if (next == BP_COUNT) {                 // the count accumulates into the slots
        s.slots[t].active = 0;
        s.slots[t].max_height = 0;
    }
}

// The work lists of the step, one workgroup per 256 candidates of a member.
__global__ void __launch_bounds__(kBlock)
k_batch_list(BatchDev *T, int tw, int th, int tj)
{
    const int64_t wg = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int ng = T->ng;
    if (wg >= T->list_off[ng]) return;
    int lo = 0, hi = ng - 1;                 // largest member with list_off <= wg
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T->list_off[mid] <= wg) lo = mid;
        else hi = mid - 1;
    }
    const MemberCtl &c = T->ctl[lo];
    const int phase = c.phase;
    if (phase != BP_RELAX && phase != BP_PUSH && phase != BP_RELABEL && phase != BP_SWEEP) return;
    const Graph s = T->graphs[lo];
    const int64_t id = (wg - T->list_off[lo]) * kBlock + threadIdx.x;
    bool want = false;
    if (phase == BP_RELAX) {
        if (id < c.tiles) {
            const int pass = c.pass;
            if (pass == 1) {
                want = true;
            } else {
                const int ntx = (s.W + tw - 1) / tw, nty = (s.H + th - 1) / th, ntz = (s.J + tj - 1) / tj;
                const int bx = (int)(id % ntx), by = (int)((id / ntx) % nty), bz = (int)(id / ((int64_t)ntx * nty));
                for (int q = 0; q < 27 && !want; ++q) {
                    const int tz = bz + q / 9 - 1, ty = by + (q / 3) % 3 - 1, tx = bx + q % 3 - 1;
                    if (tz >= 0 && tz < ntz && ty >= 0 && ty < nty && tx >= 0 && tx < ntx)
                        want = (s.stamps[(tz * nty + ty) * ntx + tx] >> 1) == pass - 1;
                }
            }
        }
        block_append(want, (int32_t)id, s.tlist, &s.hdr->lists[2]);
    } else {
        if (id < c.blocks) {
            const uint32_t a = *(const uint32_t *)(s.bact + 4 * id);
            const uint32_t f = phase == BP_PUSH ? 0u : *(const uint32_t *)(s.binf + 4 * id);
            want = (a | f) != 0u;
        }
        block_append(want, (int32_t)id, s.blist, &s.hdr->lists[0]);
    }
}

// Units of every member in this step and their prefix offsets, per kind.
__global__ void __launch_bounds__(kMaxBatch)
k_batch_scan(BatchDev *T)
{
    __shared__ int sc[3][kMaxBatch];
    const int g = threadIdx.x, ng = T->ng;
    int u = 0, kind = BK_FULL, live = 0;
    if (g < ng) {
        MemberCtl &c = T->ctl[g];
        const Graph &s = T->graphs[g];
        switch (c.phase) {
        case BP_SEED: case BP_COUNT: case BP_MERGE: u = c.blocks; break;
        case BP_RELAX: u = s.hdr->lists[2]; break;
        case BP_PUSH: case BP_RELABEL: case BP_SWEEP: u = s.hdr->lists[0]; break;
        default: u = 0;
        }
        kind = batch_kind(c.phase);
        // A sweep whose list holds more than half of the member's blocks
        // runs over every block in index order instead: a block then tests
        // its flags when it runs and takes flow pushed into it earlier in the
        // same sweep, as one workgroup per block does, where a list fixed
        // before the sweep leaves it for the next one.
        c.dense = kind == BK_SWEEP && 2 * u > c.blocks;
        if (c.dense) u = c.blocks;
        c.units = u;
        live = c.phase != BP_DONE;
    }
    for (int k = 0; k < 3; ++k) sc[k][g] = kind == k ? u : 0;
    __syncthreads();
    for (int off = 1; off < kMaxBatch; off <<= 1) {      // inclusive scans
        int v[3];
        for (int k = 0; k < 3; ++k) v[k] = g >= off ? sc[k][g - off] : 0;
        __syncthreads();
        for (int k = 0; k < 3; ++k) sc[k][g] += v[k];
        __syncthreads();
    }
    for (int k = 0; k < 3; ++k) {
        if (g < ng) T->unit_off[k][g + 1] = sc[k][g];
        if (g == 0) {
            T->unit_off[k][0] = 0;
            T->total[k] = ng > 0 ? sc[k][ng - 1] : 0;
        }
    }
    const int nlive = block_sum(live);
    if (g == 0) {
        T->live = nlive;
        T->step++;
    }
}

// The member a unit of a kind belongs to: the largest g with off[g] <= u
// (that member has units, since u < off[ng]).
__device__ inline int batch_member(const int32_t *off, int ng, int u)
{
    int lo = 0, hi = ng - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Every block of the members in a seeding, counting or merging step.
__global__ void __launch_bounds__(kBlock)
k_batch_full(const BatchDev *__restrict__ T)
{
    const int total = T->total[BK_FULL], ng = T->ng;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int g = __builtin_amdgcn_readfirstlane(batch_member(T->unit_off[BK_FULL], ng, u));
        const Graph &s = T->graphs[g];          // fields load as needed (a copy held every one)
        const int k = __builtin_amdgcn_readfirstlane(u - T->unit_off[BK_FULL][g]);
        switch (T->ctl[g].phase) {
        case BP_SEED:
            mask_blk(s, k, 0);
            seed_blk(s, k, 0);
            break;
        case BP_COUNT: count_blk(s, k); break;
        case BP_MERGE: merge_blk(s, k); break;
        default: break;
        }
        __syncthreads();                     // the count's shared memory is reused by the next unit
    }
}

// The listed tiles of the members in a relaxation pass.
template <int TW, int TH, int TJ>
__global__ void __launch_bounds__(kBlock)
k_batch_relax(const BatchDev *__restrict__ T)
{
    const int total = T->total[BK_RELAX], ng = T->ng;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int g = __builtin_amdgcn_readfirstlane(batch_member(T->unit_off[BK_RELAX], ng, u));
        const Graph &s = T->graphs[g];          // fields load as needed (a copy held every one)
        const int k = u - T->unit_off[BK_RELAX][g];
        relax_blk<TW, TH, TJ, true>(s, __builtin_amdgcn_readfirstlane(s.tlist[k]), 0, relax_rounds(T->local_iters, s),
                              __builtin_amdgcn_readfirstlane(T->ctl[g].pass));
        __syncthreads();
    }
}

// The listed blocks of the members in a push, relabel or fused sweep.
__global__ void __launch_bounds__(kBlock)
k_batch_sweeps(const BatchDev *__restrict__ T)
{
    const int total = T->total[BK_SWEEP], ng = T->ng;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int g = __builtin_amdgcn_readfirstlane(batch_member(T->unit_off[BK_SWEEP], ng, u));
        const Graph &s = T->graphs[g];          // fields load as needed (a copy held every one)
        const int k = u - T->unit_off[BK_SWEEP][g];
        const int64_t lb = T->ctl[g].dense ? k : __builtin_amdgcn_readfirstlane(s.blist[k]);
        switch (T->ctl[g].phase) {
        case BP_PUSH: push_blk(s, lb); break;
        case BP_RELABEL: relabel_blk(s, lb); break;
        case BP_SWEEP: sweep_blk(s, lb); break;
        default: break;
        }
    }
}

using BatchWorkFn = void (*)(const BatchDev *__restrict__);   // the relaxation kernel of a tile shape

// Relaxation tiles the batch engine is compiled for (the autotuner's candidates).
#define GC_BATCH_SHAPES(X) X(8, 8, 16) X(16, 8, 16) X(8, 8, 32) X(16, 16, 8)

BatchWorkFn batch_work_kernel(int tw, int th, int tj)
{
#define GC_BATCH_CASE(a, b, c) \
    if (tw == a && th == b && tj == c) return k_batch_relax<a, b, c>;
    GC_BATCH_SHAPES(GC_BATCH_CASE)
#undef GC_BATCH_CASE
    return nullptr;
}

// Steps per replay: the host reads the members' records once per this many
// steps (a member that finishes early in a replay waits for its end).
constexpr int kBatchSteps = 32;

}  // namespace

struct gc_batch {
    struct Member {
        gc_graph g;
        Graph s;
        int64_t tag;
        bool reported = false;
    };
    BatchDev *dev = nullptr;
    Opts opt{};
    BatchWorkFn work = nullptr;
    std::vector<Member> mem;
    std::vector<MemberCtl> ctl;        // host copy of the members' records
    std::vector<char> host;            // staging copy of the table
    bool dirty = true;
    int64_t list_wgs = 0;
    hipGraphExec_t exec = nullptr;
    hipStream_t exec_stream = nullptr;
    MemberCtl *pinned = nullptr;       // landing buffer of the records' read-back
    int launched = 0;                  // members whose records the read-back in flight covers
};

namespace {

MemberCtl member_init(const gc_batch *b, const Graph &s)
{
    MemberCtl c;
    memset(&c, 0, sizeof(c));
    c.phase = BP_INIT;
    c.fused = sweep_fused(b->opt) ? 1 : 0;
    c.blocks = (int32_t)grid_for(s.N);
    c.tiles = (int32_t)relax_tiles(s, b->opt);
    return c;
}

void batch_drop_graph(gc_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->exec_stream = nullptr;
}

// Writes the table: members, their records as last read back, offsets.
int batch_upload(gc_batch *b, hipStream_t st)
{
    BatchDev *h = (BatchDev *)b->host.data();
    const int ng = (int)b->mem.size();
    memset(h, 0, sizeof(BatchDev));
    h->ng = ng;
    h->live = ng;
    h->period = b->opt.period;
    h->max_sweeps = b->opt.max_sweeps;
    h->local_iters = b->opt.local_iters;
    h->flags = b->opt.flags;
    h->relabel_passes = b->opt.relabel_passes;
    h->list_off[0] = 0;
    for (int g = 0; g < ng; ++g) {
        h->graphs[g] = b->mem[g].s;
        h->ctl[g] = b->ctl[g];
        const int64_t cand = std::max<int64_t>(b->ctl[g].blocks, b->ctl[g].tiles);
        h->list_off[g + 1] = h->list_off[g] + (int32_t)((cand + kBlock - 1) / kBlock);
    }
    b->list_wgs = h->list_off[ng];
    if (!hip_ok(hipMemcpyAsync(b->dev, h, sizeof(BatchDev), hipMemcpyHostToDevice, st))) return GC_E_HIP;
    if (!hip_ok(hipStreamSynchronize(st))) return GC_E_HIP;   // the staging copy is reused
    b->dirty = false;
    return GC_OK;
}

void launch_batch_steps(gc_batch *b, hipStream_t st, int steps)
{
    const int ng = (int)b->mem.size();
    for (int i = 0; i < steps; ++i) {
        hipLaunchKernelGGL(k_batch_phase, dim3(ng), dim3(kSlots), 0, st, b->dev);
        hipLaunchKernelGGL(k_batch_list, batch_grid(b->list_wgs), dim3(kBlock), 0, st, b->dev,
                           b->opt.tw, b->opt.th, b->opt.tj);
        hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(kMaxBatch), 0, st, b->dev);
        hipLaunchKernelGGL(k_batch_full, dim3(resident_grid(k_batch_full)), dim3(kBlock), 0, st,
                           (const BatchDev *)b->dev);
        hipLaunchKernelGGL(b->work, dim3(resident_grid(b->work)), dim3(kBlock), 0, st, (const BatchDev *)b->dev);
        hipLaunchKernelGGL(k_batch_sweeps, dim3(resident_grid(k_batch_sweeps)), dim3(kBlock), 0, st,
                           (const BatchDev *)b->dev);
    }
}

}  // namespace

GC_API size_t gc_batch_footprint_bytes(void) { return align256(sizeof(BatchDev)); }

GC_API int gc_batch_create(void *dev_table, size_t dev_bytes, const gc_solve_opts *o,
                           gc_batch **out)
{
    if (!dev_table || !out || ((uintptr_t)dev_table & 255) != 0) return GC_E_ARG;
    if (dev_bytes < gc_batch_footprint_bytes()) return GC_E_WORKSPACE;
    Opts opt = resolve(o);
    int rc = check_opts(opt);
    if (rc != GC_OK) return rc;
    BatchWorkFn work = batch_work_kernel(opt.tw, opt.th, opt.tj);
    if (!work) return GC_E_ARG;
    gc_batch *b = new (std::nothrow) gc_batch();
    if (!b) return GC_E_ARG;
    b->dev = (BatchDev *)dev_table;
    b->opt = opt;
    b->work = work;
    b->host.assign(sizeof(BatchDev), 0);
    // pinned, so that the read-back does not block the host thread (a
    // pageable destination is copied synchronously)
    if (hipHostMalloc((void **)&b->pinned, kMaxBatch * sizeof(MemberCtl), hipHostMallocDefault) != hipSuccess)
        b->pinned = nullptr;
    *out = b;
    return GC_OK;
}

GC_API int gc_batch_destroy(gc_batch *b)
{
    if (!b) return GC_E_ARG;
    batch_drop_graph(b);
    if (b->pinned) (void)hipHostFree(b->pinned);
    delete b;
    return GC_OK;
}

GC_API int gc_batch_members(const gc_batch *b)
{
    if (!b) return 0;
    int n = 0;
    for (const auto &m : b->mem) n += m.reported ? 0 : 1;
    return n;
}

GC_API int gc_batch_add(gc_batch *b, const gc_graph *g, int64_t tag)
{
    if (!b) return GC_E_ARG;
    int rc = graph_check(g);
    if (rc != GC_OK) return rc;
    if (g->compact) return GC_E_ARG;           // the batch kernels take the lattice topology
    if (gc_batch_members(b) >= kMaxBatch) return GC_E_ARG;
    gc_batch::Member m;
    m.g = *g;
    m.s = view(g);
    m.tag = tag;
    b->mem.push_back(m);
    b->ctl.push_back(member_init(b, m.s));
    b->dirty = true;
    return GC_OK;
}

namespace {

// Reports finished members not yet reported (at most max_done in total).
void batch_report(gc_batch *b, int64_t *done_tags, gc_solve_stats *done_stats, int32_t max_done,
                  int32_t *n_done)
{
    for (size_t i = 0; i < b->mem.size() && *n_done < max_done; ++i) {
        gc_batch::Member &m = b->mem[i];
        if (m.reported) continue;
        if (m.s.N == 0) { b->ctl[i].phase = BP_DONE; b->ctl[i].status = GC_OK; }   // empty: done at once
        if (b->ctl[i].phase != BP_DONE) continue;
        const MemberCtl &c = b->ctl[i];
        done_tags[*n_done] = m.tag;
        if (done_stats) {
            gc_solve_stats &o = done_stats[*n_done];
            memset(&o, 0, sizeof(o));
            o.sweeps = c.sweeps;
            o.global_relabels = c.relabels;
            o.bfs_passes = c.passes;
            o.active_last = c.active;
            o.pushes = c.pushes;
            o.active_visits = c.visits;
        }
        ++*n_done;
        m.reported = true;
    }
}

// First half of a round: reports what already finished, writes the table
// again if members joined, queues the steps and the records' read-back on
// `st`, and returns without waiting (b->launched = 0 when nothing runs).
int batch_round_launch(gc_batch *b, hipStream_t st, int64_t *done_tags, gc_solve_stats *done_stats,
                       int32_t max_done, int32_t *n_done)
{
    b->launched = 0;
    batch_report(b, done_tags, done_stats, max_done, n_done);
    int live = 0;
    for (size_t i = 0; i < b->mem.size(); ++i) live += (!b->mem[i].reported && b->ctl[i].phase != BP_DONE);
    if (live == 0) return GC_OK;
    // a member joined: drop the reported ones and write the table again
    if (b->dirty) {
        size_t k = 0;
        for (size_t i = 0; i < b->mem.size(); ++i)
            if (!b->mem[i].reported) { b->mem[k] = b->mem[i]; b->ctl[k] = b->ctl[i]; ++k; }
        b->mem.resize(k);
        b->ctl.resize(k);
        batch_drop_graph(b);
        int rc = batch_upload(b, st);
        if (rc != GC_OK) return rc;
    }
    const int ng = (int)b->mem.size();
    if (st != nullptr && !b->exec) {
        hipGraph_t g = nullptr;
        if (!hip_ok(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal))) return GC_E_HIP;
        launch_batch_steps(b, st, kBatchSteps);
        if (!hip_ok(hipStreamEndCapture(st, &g))) return GC_E_HIP;
        const bool ok = hip_ok(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        if (!ok) { b->exec = nullptr; return GC_E_HIP; }
        b->exec_stream = st;
    }
    if (b->exec && b->exec_stream == st) {
        if (!hip_ok(hipGraphLaunch(b->exec, st))) return GC_E_HIP;
    } else {
        launch_batch_steps(b, st, kBatchSteps);
    }
    if (!hip_ok(hipGetLastError())) return GC_E_HIP;
    void *dst = b->pinned ? (void *)b->pinned : (void *)b->ctl.data();
    if (!hip_ok(hipMemcpyAsync(dst, b->dev->ctl, (size_t)ng * sizeof(MemberCtl), hipMemcpyDeviceToHost, st)))
        return GC_E_HIP;
    b->launched = ng;
    return GC_OK;
}

// Second half: waits for the read-back and reports the members it shows finished.
int batch_round_collect(gc_batch *b, hipStream_t st, int64_t *done_tags, gc_solve_stats *done_stats,
                        int32_t max_done, int32_t *n_done)
{
    if (b->launched == 0) return GC_OK;
    if (!hip_ok(hipStreamSynchronize(st))) return GC_E_HIP;
    if (b->pinned) memcpy(b->ctl.data(), b->pinned, (size_t)b->launched * sizeof(MemberCtl));
    b->launched = 0;
    batch_report(b, done_tags, done_stats, max_done, n_done);
    return GC_OK;
}

}  // namespace

GC_API int gc_batch_round(gc_batch *b, void *stream, int64_t *done_tags, gc_solve_stats *done_stats,
                          int32_t max_done, int32_t *n_done)
{
    if (!b || !n_done || (max_done > 0 && !done_tags)) return GC_E_ARG;
    *n_done = 0;
    hipStream_t st = (hipStream_t)stream;
    int rc = batch_round_launch(b, st, done_tags, done_stats, max_done, n_done);
    if (rc != GC_OK) return rc;
    return batch_round_collect(b, st, done_tags, done_stats, max_done, n_done);
}

namespace {

// Batch engines driven from this thread: the graphs, largest first, are
// dealt to up to kBatchEngines engines, each on its own stream (the first on
// the caller's), refilled as members finish.  Every round of every engine is
// queued before any is waited for, so one engine's steps run while another
// is between rounds and each engine's step boundaries are filled by the
// other's launches.  dev_bytes holds one table per engine.
constexpr int kBatchEngines = GC_BATCH_ENGINES;

int solve_batch_merged(gc_graph *const *gs, int32_t n, void *dev_table, size_t dev_bytes,
                       const gc_solve_opts *o, gc_solve_stats *stats, void *stream)
{
    const size_t table = gc_batch_footprint_bytes();
    const int ne = (int)std::max<size_t>(1, std::min<size_t>({(size_t)kBatchEngines, (size_t)n,
                                                              dev_bytes / table}));
    hipStream_t st0 = (hipStream_t)stream;
    std::vector<gc_batch *> eng(ne, nullptr);
    std::vector<hipStream_t> sts(ne, st0);
    hipEvent_t start = nullptr, fin = nullptr;
    int rc = GC_OK;
    auto cleanup = [&]() {
        for (int e = 0; e < ne; ++e) {
            if (eng[e]) gc_batch_destroy(eng[e]);
            if (e > 0 && sts[e]) (void)hipStreamDestroy(sts[e]);
        }
        if (start) (void)hipEventDestroy(start);
        if (fin) (void)hipEventDestroy(fin);
    };
    for (int e = 0; e < ne && rc == GC_OK; ++e)
        rc = gc_batch_create((char *)dev_table + e * table, table, o, &eng[e]);
    if (rc == GC_OK && ne > 1) {
        // the other engines start after what the caller queued on its stream
        if (!hip_ok(hipEventCreateWithFlags(&start, hipEventDisableTiming)) ||
            !hip_ok(hipEventRecord(start, st0)))
            rc = GC_E_HIP;
        for (int e = 1; e < ne && rc == GC_OK; ++e) {
            sts[e] = nullptr;
            if (!hip_ok(hipStreamCreateWithFlags(&sts[e], hipStreamNonBlocking)) ||
                !hip_ok(hipStreamWaitEvent(sts[e], start, 0)))
                rc = GC_E_HIP;
        }
    }
    if (rc != GC_OK) { cleanup(); return rc; }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return node_count(&gs[a]->p) > node_count(&gs[b]->p);
    });
    const auto t0 = std::chrono::steady_clock::now();
    int next = 0, done = 0, status = GC_OK;
    std::vector<int64_t> tags(kMaxBatch);
    std::vector<gc_solve_stats> st_out(kMaxBatch);
    auto take = [&](int e, int32_t nd) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int i = 0; i < nd; ++i) {
            st_out[i].done_ms = ms;
            if (stats) stats[tags[i]] = st_out[i];
            if (st_out[i].active_last != 0) status = GC_E_NOT_CONVERGED;
        }
        done += nd;
    };
    // deal the graphs to the engines in turn (largest first), as far as they hold
    for (int e = 0; next < n && rc == GC_OK; e = (e + 1) % ne) {
        bool room = false;
        for (int f = 0; f < ne; ++f) room = room || gc_batch_members(eng[f]) < kMaxBatch;
        if (!room) break;
        if (gc_batch_members(eng[e]) >= kMaxBatch) continue;
        if ((rc = gc_batch_add(eng[e], gs[order[next]], order[next])) == GC_OK) ++next;
    }
    for (int e = 0; e < ne && rc == GC_OK; ++e) {
        int32_t nd = 0;
        rc = batch_round_launch(eng[e], sts[e], tags.data(), st_out.data(), kMaxBatch, &nd);
        if (rc == GC_OK) take(e, nd);
    }
    // each engine is collected and relaunched in turn, so its next round is
    // queued as soon as its last one ends while the others keep running
    while (done < n && rc == GC_OK) {
        for (int e = 0; e < ne && rc == GC_OK; ++e) {
            int32_t nd = 0;
            rc = batch_round_collect(eng[e], sts[e], tags.data(), st_out.data(), kMaxBatch, &nd);
            if (rc != GC_OK) break;
            take(e, nd);
            while (next < n && gc_batch_members(eng[e]) < kMaxBatch) {   // refill
                if ((rc = gc_batch_add(eng[e], gs[order[next]], order[next])) != GC_OK) break;
                ++next;
            }
            if (rc != GC_OK) break;
            nd = 0;
            rc = batch_round_launch(eng[e], sts[e], tags.data(), st_out.data(), kMaxBatch, &nd);
            if (rc == GC_OK) take(e, nd);
        }
    }
    if (rc == GC_OK && ne > 1) {
        // the caller's stream sees the other engines' work as done
        if (!hip_ok(hipEventCreateWithFlags(&fin, hipEventDisableTiming))) rc = GC_E_HIP;
        for (int e = 1; e < ne && rc == GC_OK; ++e)
            if (!hip_ok(hipEventRecord(fin, sts[e])) || !hip_ok(hipStreamWaitEvent(st0, fin, 0))) rc = GC_E_HIP;
        if (rc == GC_OK && !hip_ok(hipStreamSynchronize(st0))) rc = GC_E_HIP;
    }
    cleanup();
    return rc != GC_OK ? rc : status;
}

// Concurrent lanes: worker threads with their own streams take the graphs,
// largest first, and solve each as maxflow_solve does.
int solve_batch_lanes(gc_graph *const *gs, int32_t n, const gc_solve_opts *o, gc_solve_stats *stats,
                      void *stream)
{
    int dev = 0;
    if (!hip_ok(hipGetDevice(&dev))) return GC_E_HIP;
    hipEvent_t start = nullptr;
    if (!hip_ok(hipEventCreateWithFlags(&start, hipEventDisableTiming))) return GC_E_HIP;
    if (!hip_ok(hipEventRecord(start, (hipStream_t)stream))) { (void)hipEventDestroy(start); return GC_E_HIP; }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return node_count(&gs[a]->p) > node_count(&gs[b]->p);
    });
    const auto t0 = std::chrono::steady_clock::now();
    std::atomic<int> next{0}, error{GC_OK}, unconverged{0};
    auto worker = [&]() {
        int rc = hip_ok(hipSetDevice(dev)) ? GC_OK : GC_E_HIP;
        hipStream_t st = nullptr;
        if (rc == GC_OK && !hip_ok(hipStreamCreateWithFlags(&st, hipStreamNonBlocking))) rc = GC_E_HIP;
        if (rc == GC_OK && !hip_ok(hipStreamWaitEvent(st, start, 0))) rc = GC_E_HIP;
        while (rc == GC_OK && error.load() == GC_OK) {
            const int k = next.fetch_add(1);
            if (k >= n) break;
            const int i = order[k];
            gc_solve_stats one;
            memset(&one, 0, sizeof(one));
            const int r = maxflow_solve(gs[i], o, &one, st);   // returns with its stream drained
            one.done_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (stats) stats[i] = one;
            if (r == GC_E_NOT_CONVERGED) unconverged = 1;
            else if (r != GC_OK) rc = r;
        }
        if (st) {
            if (!hip_ok(hipStreamSynchronize(st)) && rc == GC_OK) rc = GC_E_HIP;
            (void)hipStreamDestroy(st);
        }
        if (rc != GC_OK) {
            int expect = GC_OK;
            error.compare_exchange_strong(expect, rc);
        }
    };
    const int lanes = n < GC_BATCH_LANES ? n : GC_BATCH_LANES;
    std::vector<std::thread> th;
    th.reserve(lanes);
    for (int l = 0; l < lanes; ++l) th.emplace_back(worker);
    for (std::thread &t : th) t.join();
    (void)hipEventDestroy(start);
    if (error.load() != GC_OK) return error.load();
    return unconverged.load() ? GC_E_NOT_CONVERGED : GC_OK;
}

}  // namespace

GC_API int maxflow_solve_batch(gc_graph *const *gs, int32_t n, void *dev_table, size_t dev_bytes,
                               const gc_solve_opts *o, gc_solve_stats *stats, void *stream)
{
    if (n < 0 || (n > 0 && !gs)) return GC_E_ARG;
    for (int i = 0; i < n; ++i) {
        int rc = graph_check(gs[i]);
        if (rc != GC_OK) return rc;
    }
    const Opts opt = resolve(o);
    int rc = check_opts(opt);
    if (rc != GC_OK) return rc;
    if (n == 0) return GC_OK;
    if (opt.flags & GC_OPT_BATCH_MERGED) return solve_batch_merged(gs, n, dev_table, dev_bytes, o, stats, stream);
    return solve_batch_lanes(gs, n, o, stats, stream);
}

GC_API int gc_graph_state(const gc_graph *g, int32_t *excess, int32_t *words, void *stream)
{
    int rc = graph_check(g);
    if (rc != GC_OK) return rc;
    if (!excess || !words || g->compact) return GC_E_ARG;
    const Graph s = view(g);
    if (s.N == 0) return GC_OK;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = (size_t)s.N * sizeof(int32_t);
    if (!hip_ok(hipMemcpyAsync(excess, s.ex, bytes, hipMemcpyDeviceToDevice, st))) return GC_E_HIP;
    const int32_t *src[7] = {s.rd, s.re, s.rs, s.rem, s.rep, s.rsm, s.rsp};
    for (int i = 0; i < 7; ++i)
        if (!hip_ok(hipMemcpyAsync(words + (size_t)i * s.N, src[i], bytes, hipMemcpyDeviceToDevice, st)))
            return GC_E_HIP;
    return GC_OK;
}

// The read-out of extract_labels (rb as for solve_graph).
static int extract_graph(const gc_graph *g, const int32_t *cost, int32_t *labels, int64_t *result,
                         hipStream_t st, HeaderRead *rb)
{
    int rc;
    Graph s = view(g);
    const gc_problem &p = g->p;
    Opts opt = resolve(nullptr);
    Launcher L{st, false, {}};
    L.rb = rb;
    int passes = 0;
    if (s.N > 0) {
        const unsigned grid = grid_for(s.N);
        hipLaunchKernelGGL(mask_kernel(s), dim3(grid), dim3(kBlock), 0, st, s, 1);
        hipLaunchKernelGGL(k_seed<Graph>, dim3(grid), dim3(kBlock), 0, st, s, 1);
        if (!hip_ok(hipGetLastError())) return GC_E_HIP;
        if ((rc = relax_to_fixpoint(s, 1, opt, L, &passes)) != GC_OK) return rc;
    }
    hipLaunchKernelGGL(k_zero_result, dim3(1), dim3(64), 0, st, result, s.hdr);
    hipLaunchKernelGGL(k_zero_slots, dim3(1), dim3(kSlots), 0, st, s.slots, 2);
    if (s.plane > 0) {
        hipLaunchKernelGGL(k_labels, dim3(grid_for(s.plane)), dim3(kBlock), 0, st, s, labels, 1);
        hipLaunchKernelGGL(k_energy, dim3(grid_for(s.plane)), dim3(kBlock), 0, st, cost, labels,
                           p.width, p.height, p.labels, p.penalty_h, p.inhibit_h, p.penalty_v,
                           p.inhibit_v, s.slots);
    }
    if (s.N > 0)
        hipLaunchKernelGGL(k_deficit, dim3(grid_for(s.N)), dim3(kBlock), 0, st, s);
    hipLaunchKernelGGL(k_fold_slots, dim3(1), dim3(kSlots), 0, st, s.slots, s.hdr, 2, result);
    if (!hip_ok(hipGetLastError())) return GC_E_HIP;
    int32_t perr = 0;
    if ((rc = read_i32(&s.hdr->prefix_err, &perr, st)) != GC_OK) return rc;
    return (perr & kCostErr) ? GC_E_CAP_OVERFLOW : perr ? GC_E_PREFIX : GC_OK;
}

GC_API int extract_labels(const gc_graph *g, const int32_t *cost, int32_t *labels,
                          int64_t *result, void *stream)
{
    int rc = graph_check(g);
    if (rc != GC_OK) return rc;
    if (!cost || !labels || !result) return GC_E_ARG;
    return extract_graph(g, cost, labels, result, (hipStream_t)stream, nullptr);
}

// ---------------------------------------------------------------------------
// The path without allocation: the cost volume and the graph live in a
// file-scope device array.  In host code `scratch` names a host-side stand-in,
// not device memory: only the address hipGetSymbolAddress returns for the
// current device may reach a kernel or a copy.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[GC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void *g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current), or null when the lookup failed.
void *scratch_address(int dev)
{
    std::call_once(g_scratch_once[dev], [dev] {
        void *ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
    });
    if (!g_scratch_ptr[dev]) t_last_hip = (int)g_scratch_err[dev];
    return g_scratch_ptr[dev];
}

}  // namespace

GC_API size_t gc_solve_pair_static_bytes(const gc_problem *p)
{
    if (gc_problem_check(p) != GC_OK) return 0;
    const size_t cost = align256((size_t)p->labels * p->height * p->width * sizeof(int32_t));
    return cost + gc_graph_footprint_bytes(p);
}

GC_API int gc_solve_pair_static(const uint8_t *left, const uint8_t *right, const gc_problem *p,
                                const gc_solve_opts *o, int32_t *labels, int64_t *result,
                                gc_solve_stats *stats, void *stream)
{
    int rc = gc_problem_check(p);
    if (rc != GC_OK) return rc;
    if (!left || !right || !labels || !result) return GC_E_ARG;
    Opts opt = resolve(o);
    if ((rc = check_opts(opt)) != GC_OK) return rc;
    // kernel timing creates events, captured sweeps instantiate graphs
    if (opt.flags & (GC_OPT_TIME_KERNELS | GC_OPT_SWEEP_GRAPH)) return GC_E_ARG;
    const size_t need = gc_solve_pair_static_bytes(p);
    if (need > sizeof(scratch)) return GC_E_WORKSPACE;
    int dev = 0;
    if (!hip_ok(hipGetDevice(&dev))) return GC_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return GC_E_ARG;
    unsigned char *base = (unsigned char *)scratch_address(dev);
    if (!base) return GC_E_HIP;
    hipStream_t st = (hipStream_t)stream;
    int32_t *cost = (int32_t *)base;
    const size_t cost_bytes = align256((size_t)p->labels * p->height * p->width * sizeof(int32_t));
    gc_graph g;
    if ((rc = stereo_cost_volume(left, right, p, cost, stream)) != GC_OK) return rc;
    if ((rc = graph_build(p, cost, base + cost_bytes, sizeof(scratch) - cost_bytes, &g, stream)) != GC_OK)
        return rc;
    HeaderRead rb;                     // pageable: pinned memory would be an allocation
    if ((rc = solve_graph(&g, opt, stats, st, &rb)) != GC_OK) return rc;
    return extract_graph(&g, cost, labels, result, st, &rb);
}
