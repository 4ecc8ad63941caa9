"""Runtime above the C ABI: autotuner, batched workload runner and the
continuous-batching serving loop.

Orchestration only: every step of the path (cost volume, graph build,
max-flow, cut read-out) runs in the HIP library through ``gazecut``; the
batch engine that schedules graphs round by round is native (``gc_batch_*``).
PyTorch provides device memory and streams.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import gazecut as gc
from . import scenegen as sg


# ---------------------------------------------------------------------------
# Items of work
# ---------------------------------------------------------------------------

@dataclass
class Item:
    """One stereo pair resident on the device, with its graph workspace."""
    tag: int
    spec: sg.SceneSpec
    left: object                 # uint8 [h][w] device tensor
    right: object
    p: gc.GcProblem
    cost: object = None          # int32 [m][h][w]
    ws: object = None            # uint8 workspace
    graph: gc.Graph | None = None
    labels: object = None
    result: object = None        # int64 [2]
    energy: int = 0
    flow: int = 0
    stats: dict = field(default_factory=dict)
    t_done: float = 0.0

    @property
    def footprint(self) -> int:
        return gc.footprint_bytes(self.p) + 4 * self.p.labels * self.p.height * self.p.width


def make_item(tag, spec: sg.SceneSpec, pair: sg.Pair, lam=1, device="cuda") -> Item:
    """An item whose images are copied to `device` now; with device=None they
    stay on the host until prepare() copies them on its stream."""
    import torch
    p = gc.problem(spec.w, spec.h, spec.m, spec.cap, lam, spec.inhibit)
    if device is None:
        return Item(tag, spec, pair.left, pair.right, p)
    return Item(tag, spec, torch.from_numpy(pair.left).to(device),
                torch.from_numpy(pair.right).to(device), p)


def prepare(item: Item, stream=None):
    """Allocates device buffers, computes the cost volume and builds the graph."""
    import torch
    if isinstance(item.left, np.ndarray):
        item.left = torch.from_numpy(item.left).cuda()
        item.right = torch.from_numpy(item.right).cuda()
    dev = item.left.device
    p = item.p
    if item.cost is None:
        item.cost = torch.empty((p.labels, p.height, p.width), dtype=torch.int32, device=dev)
        item.ws = torch.empty(gc.footprint_bytes(p), dtype=torch.uint8, device=dev)
        item.labels = torch.empty((p.height, p.width), dtype=torch.int32, device=dev)
        item.result = torch.zeros(2, dtype=torch.int64, device=dev)
    gc.stereo_cost_volume(item.left, item.right, p, item.cost, stream)
    item.graph = gc.graph_build(p, item.cost, item.ws, stream)


def finish(item: Item, stream=None):
    gc.extract_labels(item.graph, item.cost, item.labels, item.result, stream)
    r = item.result.cpu().tolist()
    item.energy, item.flow = int(r[0]), int(r[1])


def release(item: Item):
    item.cost = item.ws = item.graph = None


# ---------------------------------------------------------------------------
# Autotuner: relaxation tile shape and global-relabel period
# ---------------------------------------------------------------------------

TILE_CANDIDATES = ((8, 8, 16), (16, 8, 16), (8, 8, 32), (16, 16, 8))
PERIOD_CANDIDATES = (0, 24, 32, 64)   # 0: by depth
SWEEP_CANDIDATES = (0, gc.GC_OPT_SPLIT_SWEEP)   # fused (the default), split


def autotune(items, tiles=TILE_CANDIDATES, periods=PERIOD_CANDIDATES, sweeps=SWEEP_CANDIDATES,
             stream=None, use_graph=False, extra_flags=0):
    """Times one batched solve of `items` per (tile, period, sweep kind)
    candidate and returns (best options, [(tile, period, sweep flags,
    seconds)]).  The items' graphs are rebuilt in place before every trial,
    so the trials solve the same graphs.  extra_flags selects the engine
    (GC_OPT_BATCH_MERGED: the batch engine; none: concurrent lanes)."""
    import torch
    base = (gc.GC_OPT_SWEEP_GRAPH if use_graph else 0) | extra_flags
    table = torch.empty(gc.GC_BATCH_ENGINES * gc.batch_footprint_bytes(), dtype=torch.uint8, device="cuda")
    trials = []
    for tile in tiles:
        for period in periods:
            for sw in sweeps:
                opts = gc.GcSolveOpts(relabel_period=period, tile_w=tile[0], tile_h=tile[1],
                                      tile_j=tile[2], flags=base | sw)
                for it in items:
                    prepare(it, stream)
                torch.cuda.synchronize()
                t = time.perf_counter()
                gc.maxflow_solve_batch([it.graph for it in items], opts, stream, table)
                torch.cuda.synchronize()
                trials.append((tile, period, sw, time.perf_counter() - t))
    tile, period, sw, _ = min(trials, key=lambda r: r[3])
    best = gc.GcSolveOpts(relabel_period=period, tile_w=tile[0], tile_h=tile[1], tile_j=tile[2],
                          flags=base | sw)
    return best, trials


# ---------------------------------------------------------------------------
# Batched workload: many uneven pairs, batched vs one pair per launch
# ---------------------------------------------------------------------------

def batch_mix(n=64, shapes=sg.BATCH_SHAPES, seed=4, base=sg.MID):
    """n seeded pairs, shapes drawn uniformly from `shapes` (W, H, labels),
    generated with the slanted-plane settings of `base`."""
    rng = np.random.default_rng([seed, n])
    picks = rng.integers(0, len(shapes), n)
    out = []
    for i, k in enumerate(picks):
        w, h, m = shapes[int(k)]
        spec = sg.spec_like(base, w, h, m)
        out.append((spec, sg.make_pair(spec, (seed, i))))
    return out


def run_one_per_launch(items, opts=None, stream=None):
    """Solves the items one after another; returns per-item completion times
    (seconds from the start) and the total."""
    import torch
    for it in items:
        prepare(it, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in items:
        st = gc.maxflow_solve(it.graph, opts, stream)
        finish(it, stream)
        it.t_done = time.perf_counter() - t0
        it.stats = st.as_dict()
    torch.cuda.synchronize()
    return [it.t_done for it in items], time.perf_counter() - t0


def run_batched(items, opts=None, stream=None):
    """Solves all items with one maxflow_solve_batch call (concurrent lanes,
    largest graphs first), then reads every item's labels.  Returns each
    item's solve completion time (from the library's clock, seconds from the
    call) and the total."""
    import torch
    for it in items:
        prepare(it, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = gc.maxflow_solve_batch([it.graph for it in items], opts, stream)
    for it, st in zip(items, sts):
        finish(it, stream)
        it.stats = st.as_dict()
        it.t_done = st.done_ms * 1e-3
    torch.cuda.synchronize()
    return [it.t_done for it in items], time.perf_counter() - t0


def run_merged(items, opts=None, stream=None):
    """Solves all items in rounds of the merged batch engine (one launch per
    phase over all members); each item's labels are read as soon as it
    leaves the batch.  Returns completion times and the total."""
    import torch
    for it in items:
        prepare(it, stream)
    torch.cuda.synchronize()
    b = gc.Batch.on_device(opts)
    by_tag = {it.tag: it for it in items}
    t0 = time.perf_counter()
    pending = list(items)
    done = 0
    while done < len(items):
        while pending and len(b) < gc.GC_BATCH_MAX_GRAPHS:
            it = pending.pop(0)
            b.add(it.graph, it.tag)
        for tag, st in b.round(stream):
            it = by_tag[tag]
            finish(it, stream)
            it.t_done = time.perf_counter() - t0
            it.stats = st.as_dict()
            done += 1
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    b.close()
    return [it.t_done for it in items], total


# ---------------------------------------------------------------------------
# Serving: continuous batching with admission by device-memory footprint
# ---------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival: float               # seconds after the start of the stream
    shape: tuple
    pool_index: int
    item: Item | None = None
    t_admit: float = 0.0
    t_done: float = 0.0


def poisson_requests(n, rate, shapes=sg.SERVE_SHAPES, pool_per_shape=2, seed=5):
    """n requests with exponential inter-arrival times at `rate` per second,
    shapes drawn uniformly; each request names a pair of a small seeded pool
    per shape (generating a fresh scene per request would cost more than the
    solve at these rates)."""
    rng = np.random.default_rng([seed, n])
    gaps = rng.exponential(1.0 / rate, n)
    arrivals = np.cumsum(gaps)
    picks = rng.integers(0, len(shapes), n)
    pools = rng.integers(0, pool_per_shape, n)
    return [Request(i, float(arrivals[i]), tuple(shapes[int(picks[i])]), int(pools[i]))
            for i in range(n)]


# Requests go to a lane by footprint: each lane is a batch engine on its own
# stream driven by its own host thread, so a small request does not wait for
# the rounds of a 1280x720x128 graph; the lanes' kernels share the GPU.  A
# lane is (footprint upper bound or None, most graphs in its batch): graphs
# that fill the GPU on their own gain nothing from sharing rounds, so the
# unbounded lane takes one at a time (a second unbounded lane was measured:
# two 1280x720x128 graphs at once share the memory bandwidth and each takes
# nearly twice as long, so latency got worse).  Lanes of equal bound may be
# listed; a request then goes to the least loaded of them.
DEFAULT_LANES = ((512 << 20, gc.GC_BATCH_MAX_GRAPHS), (2 << 30, 16), (None, 1))


class Lane:
    def __init__(self, server, index, limit, max_members, opts, device):
        import torch
        self.server = server
        self.index = index
        self.limit = limit
        self.max_members = max(1, min(int(max_members), gc.GC_BATCH_MAX_GRAPHS))
        self.opts = opts
        dev = torch.device(device)
        self.device = dev.index if dev.index is not None else torch.cuda.current_device()
        self.stream = torch.cuda.Stream(self.device)
        self.batch = gc.Batch.on_device(opts, f"cuda:{self.device}")
        self.cv = threading.Condition()
        self.inbox = []
        self.preparing = 0          # taken from the inbox, not yet in the batch
        self.live = {}
        self.rounds = 0
        self.closing = False
        self.error = None
        self.thread = threading.Thread(target=self._run, name=f"lane{index}", daemon=True)
        self.thread.start()

    def accepts(self, footprint):
        return self.limit is None or footprint <= self.limit

    def submit(self, req):
        with self.cv:
            self.inbox.append(req)
            self.cv.notify()

    def pending(self):
        """Requests submitted to this lane and not finished: waiting in the
        inbox, being prepared, or in the batch."""
        with self.cv:
            return len(self.inbox) + self.preparing + len(self.live)

    def _take_inbox(self):
        """Moves the inbox to the lane's preparation (still counted by pending)."""
        with self.cv:
            new, self.inbox = self.inbox, []
            self.preparing += len(new)
        return new

    def _went_live(self, req):
        with self.cv:
            self.preparing -= 1
            self.live[req.rid] = req

    def close(self):
        with self.cv:
            self.closing = True
            self.cv.notify()
        self.thread.join()
        self.batch.close()

    def _run(self):
        import torch
        try:
            torch.cuda.set_device(self.device)
            with torch.cuda.stream(self.stream):
                while True:
                    with self.cv:
                        while not self.inbox and not self.live and not self.closing:
                            self.cv.wait()
                        if self.closing and not self.inbox and not self.live:
                            return
                    for req in self._take_inbox():
                        prepare(req.item, self.stream)
                        self.batch.add(req.item.graph, req.rid)
                        self._went_live(req)
                    self.server._members()
                    for tag, st in self.batch.round(self.stream):
                        with self.cv:
                            req = self.live.pop(tag)
                        finish(req.item, self.stream)
                        req.item.stats = st.as_dict()
                        if self.server.keep_labels:
                            req.item.labels = req.item.labels.cpu().numpy()
                        else:
                            req.item.labels = None
                        req.t_done = self.server.clock()
                        release(req.item)
                        self.server._complete(req)
                    self.rounds += 1
        except Exception as e:                         # reported by the serving thread
            self.error = e
            self.server._complete(None)


class Server:
    """Continuous batching over the native batch engine.

    Requests go to the first lane whose footprint bound holds them and are
    admitted first come, first served within their lane while the bytes of
    live graph workspaces and cost volumes stay within `budget_bytes` and the
    lane has room (a request that has to wait holds back only later requests
    of its own lane).  A lane builds an admitted request's cost volume and graph on
    its stream and adds the graph to its running batch at the next round, so
    its work overlaps with the requests already on the GPU; finished graphs
    leave the batch, their labels are read and their memory is freed.
    """

    def __init__(self, budget_bytes, opts=None, lanes=DEFAULT_LANES, device="cuda", keep_labels=False):
        import time as _time
        self.budget = int(budget_bytes)
        self.keep_labels = keep_labels
        self.lock = threading.Condition()
        self.used = 0
        self.peak_used = 0
        self.peak_members = 0
        self.done = []
        self.t0 = _time.perf_counter()
        self.lanes = [Lane(self, i, lim, mx, opts, device) for i, (lim, mx) in enumerate(lanes)]

    def clock(self):
        return time.perf_counter() - self.t0

    @property
    def rounds(self):
        return sum(l.rounds for l in self.lanes)

    def lane_for(self, item: Item) -> Lane:
        """The lane class with the smallest bound that holds the item; among
        lanes of that class, the one with the fewest requests."""
        fit = [l for l in self.lanes if l.accepts(item.footprint)]
        if not fit:
            raise ValueError(f"no lane takes {item.footprint} B")
        bound = min(fit, key=lambda l: float("inf") if l.limit is None else l.limit).limit
        same = [l for l in fit if l.limit == bound]
        return min(same, key=lambda l: l.pending())

    def fits(self, item: Item) -> bool:
        lane = self.lane_for(item)
        with self.lock:
            return (self.used + item.footprint <= self.budget
                    and lane.pending() < lane.max_members)

    def admit(self, req: Request, item: Item, now: float):
        lane = self.lane_for(item)
        with self.lock:
            self.used += item.footprint
            self.peak_used = max(self.peak_used, self.used)
        req.item = item
        req.t_admit = now
        lane.submit(req)

    def _members(self):
        n = sum(l.pending() for l in self.lanes)
        with self.lock:
            self.peak_members = max(self.peak_members, n)

    def _complete(self, req):
        with self.lock:
            if req is not None:
                self.used -= req.item.footprint
                self.done.append(req)
            self.lock.notify_all()

    def wait(self, timeout):
        with self.lock:
            self.lock.wait(timeout)

    def check(self):
        for lane in self.lanes:
            if lane.error is not None:
                raise lane.error

    def close(self):
        for lane in self.lanes:
            lane.close()


def serve(requests, pools, budget_bytes, opts=None, lanes=DEFAULT_LANES, lam=1, keep_labels=False,
          max_wall_s=None, progress=None, progress_every=100):
    """Runs the request stream in real time.  `pools[shape][i]` is the
    (spec, pair) a request names.  Returns (completed requests, wall seconds,
    server).  With keep_labels the labels are kept as host arrays.
    `progress(n_done, seconds)` is called each time another
    `progress_every` requests have completed."""
    import torch
    srv = Server(budget_bytes, opts, lanes, keep_labels=keep_labels)
    queue = list(requests)
    qi = 0
    waiting = []                                        # arrived, not admitted, in arrival order
    srv.t0 = time.perf_counter()
    reported = 0
    try:
        while True:
            srv.check()
            with srv.lock:
                n_done = len(srv.done)
            if progress is not None and n_done >= reported + progress_every:
                reported = n_done - n_done % progress_every
                progress(n_done, srv.clock())
            if n_done == len(queue):
                break
            now = srv.clock()
            if max_wall_s is not None and now > max_wall_s:
                break
            while qi < len(queue) and queue[qi].arrival <= now:
                req = queue[qi]
                spec, pair = pools[req.shape][req.pool_index]
                item = make_item(req.rid, spec, pair, lam, device=None)
                if item.footprint > budget_bytes:
                    raise ValueError(f"request {req.rid} needs {item.footprint} B, budget {budget_bytes}")
                waiting.append((req, item))
                qi += 1
            # first come, first served within a lane class (footprint bound):
            # a request that does not fit (its lanes full or the memory
            # budget) holds back the later requests of its own class only
            blocked = set()
            still = []
            for req, item in waiting:
                lane = srv.lane_for(item)
                if lane.limit in blocked or not srv.fits(item):
                    blocked.add(lane.limit)
                    still.append((req, item))
                else:
                    srv.admit(req, item, now)
            waiting = still
            wait = 0.002
            if qi < len(queue):
                wait = max(0.0, min(wait, queue[qi].arrival - srv.clock()))
            srv.wait(wait)
    finally:
        srv.close()
    torch.cuda.synchronize()
    with srv.lock:
        done = list(srv.done)
    return done, srv.clock(), srv


def latency_summary(done):
    lat = np.array([r.t_done - r.arrival for r in done]) * 1e3
    wait = np.array([r.t_admit - r.arrival for r in done]) * 1e3
    if lat.size == 0:
        return {}
    return {"p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "mean_ms": round(float(lat.mean()), 2),
            "admission_wait_p50_ms": round(float(np.percentile(wait, 50)), 2),
            "admission_wait_p99_ms": round(float(np.percentile(wait, 99)), 2),
            # share of the mean latency spent waiting for admission (memory
            # budget or a full lane) rather than on the GPU
            "queue_share": round(float(wait.mean() / lat.mean()), 4) if lat.mean() > 0 else 0.0}
