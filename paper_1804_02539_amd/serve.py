"""Continuous-batching solve server on one GPU.

Requests (a problem description plus a right-hand side) arrive at any time.
The server keeps multigrid hierarchies resident on the device (one or more
handles per distinct problem), admits a request as soon as a handle for its
problem is idle or a new one fits in the HBM budget (evicting idle handles of
other problems least-recently-used first), and steps every running request in
lockstep through one ``igamg.Batch``: each step is one PCG iteration of every
running request, replayed as HIP graphs in which each request is an
independent branch, so requests that arrive while others are on the GPU join
the next step and their work overlaps on the device.  Hierarchy setups (host
assembly and upload) run on a worker pool while the batch keeps stepping.

The backend is injectable (``make_solver``, ``workspace_bytes``, ``batch``) so
the admission logic can be exercised without a GPU.
"""
import collections
import concurrent.futures as cf
import hashlib
import time

import numpy as np


class ServeError(RuntimeError):
    pass


def problem_key(prob, opts_tuple=()):
    """Identity of a discretised problem (geometry, topology, degree, levels)."""
    h = hashlib.sha1()
    for a in (prob.nel0, prob.geo_degree, prob.iface, prob.bc):
        h.update(np.ascontiguousarray(a, dtype=np.int64).tobytes())
    h.update(prob.flat_ctrl().tobytes())
    h.update(np.array([prob.dim, prob.degree, prob.levels], dtype=np.int64).tobytes())
    h.update(repr(opts_tuple).encode())
    return h.hexdigest()[:20]


class Request:
    _ids = iter(range(1 << 62))

    def __init__(self, problem, rhs_fn, tol=1e-8, arrival=None, key=None):
        self.id = next(Request._ids)
        self.problem = problem
        self.rhs_fn = rhs_fn          # N -> host array of length N (free dofs)
        self.tol = tol
        self.arrival = time.perf_counter() if arrival is None else arrival
        self.key = key or problem_key(problem)
        self.admitted = None
        self.done = None
        self.info = None
        self.code = None
        self.result = None            # device tensor (solution), when done
        self.n = None
        self.error = None

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


class _Handle:
    def __init__(self, key, solver, nbytes):
        self.key = key
        self.solver = solver
        self.nbytes = nbytes
        self.busy = False
        self.last_used = time.perf_counter()


class Server:
    def __init__(self, hbm_budget, *, opts=None, device="cuda:0", setup_workers=2,
                 max_active=64, handles_per_key=2, make_solver=None, workspace_bytes=None,
                 batch=None, keep_results=True):
        self.budget = int(hbm_budget)
        self.device = device
        self.max_active = max_active
        self.handles_per_key = handles_per_key
        self.keep_results = keep_results
        if make_solver is None or workspace_bytes is None or batch is None:
            from . import igamg
            self.opts = opts or igamg.default_options()
            def _setup(prob):
                import torch
                # each setup uploads on a stream of its own (never the legacy
                # default stream, so it cannot serialise against the batch)
                st = torch.cuda.Stream(device=device)
                for attempt in (0, 1):
                    try:
                        with torch.cuda.stream(st):
                            S = igamg.Solver(prob, self.opts, device=device, stream=st)
                        break
                    except torch.cuda.OutOfMemoryError:
                        # the budget fits, so the allocator's cache is holding
                        # the memory: return it to the device and try once more
                        if attempt:
                            raise
                        torch.cuda.synchronize(device)
                        torch.cuda.empty_cache()
                st.synchronize()
                return S
            make_solver = make_solver or _setup
            workspace_bytes = workspace_bytes or (lambda prob: igamg.workspace_size(prob, self.opts) + 256)
            batch = batch or igamg.Batch()
        self._make = make_solver
        self._wsbytes = workspace_bytes
        self.batch = batch
        self.pending = collections.deque()
        self.handles = collections.defaultdict(list)   # key -> [_Handle]
        self.setups = {}                                # future -> (key, nbytes)
        self.running = {}                               # slot -> (Request, _Handle)
        self.finished = []
        self.rejected = []
        self.used = 0                                   # resident + reserved bytes
        self.peak_used = 0
        self.steps = 0
        self._size_cache = {}
        self._pool = cf.ThreadPoolExecutor(max_workers=setup_workers)
        self.events = []                                # (time, kind, detail) for inspection

    # ---------------------------------------------------------------- API
    def submit(self, req):
        self.pending.append(req)
        return req

    def idle(self):
        return not self.pending and not self.running and not self.setups

    def close(self):
        self._pool.shutdown(wait=True)

    # ---------------------------------------------------------- internals
    def _nbytes(self, req):
        if req.key not in self._size_cache:
            self._size_cache[req.key] = int(self._wsbytes(req.problem))
        return self._size_cache[req.key]

    def _charge(self, nbytes):
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        assert self.used <= self.budget, "admission exceeded the HBM budget"

    def _evict_for(self, nbytes, protect_key, wanted=()):
        """Free idle handles until nbytes fit: first those no waiting request
        needs, least recently used first, the requesting problem's last."""
        if self.used + nbytes <= self.budget:
            return True
        idle = [h for hs in self.handles.values() for h in hs if not h.busy]
        idle.sort(key=lambda h: (h.key in wanted, h.key == protect_key, h.last_used))
        for h in idle:
            if self.used + nbytes <= self.budget:
                break
            self.handles[h.key].remove(h)
            self._release(h)
            self.used -= h.nbytes
            self.events.append((time.perf_counter(), "evict", h.key))
        return self.used + nbytes <= self.budget

    def _release(self, h):
        # an idle handle has no queued work left in the batch (its request was
        # retired after the batch synchronised), but the workspace memory
        # returns to the allocator, so make sure no stream still reads it
        if not self.device.startswith("cuda"):
            h.solver = None
            return
        import torch
        torch.cuda.synchronize(self.device)
        h.solver = None
        # hand the workspace back to the device at once: left in the
        # allocator's cache, a smaller workspace would later split it, and a
        # partly used segment can never be released for a large one
        torch.cuda.empty_cache()

    def _collect_setups(self):
        for fut in [f for f in self.setups if f.done()]:
            key, nbytes = self.setups.pop(fut)
            try:
                solver = fut.result()
            except Exception as e:  # setup failed: release the reservation
                self.used -= nbytes
                self.events.append((time.perf_counter(), "setup_error", f"{key}: {e}"))
                for r in [r for r in self.pending if r.key == key]:
                    r.error = e
                    r.code = getattr(e, "code", -1)
                    self.pending.remove(r)
                    self.rejected.append(r)
                continue
            self.handles[key].append(_Handle(key, solver, nbytes))
            self.events.append((time.perf_counter(), "resident", key))

    def _start(self, req, h):
        import torch
        h.busy = True
        h.last_used = time.perf_counter()
        req.n = h.solver.N
        rhs = torch.as_tensor(req.rhs_fn(req.n), dtype=torch.float64, device=self.device)
        slot = self.batch.add(h.solver, rhs, tol=req.tol)
        req.admitted = time.perf_counter()
        self.running[slot] = (req, h)

    def _admit(self):
        # first every request whose problem is resident and idle: a hierarchy
        # that has just been set up must serve its request before any other
        # problem may evict it (else two problems can evict each other forever)
        for req in list(self.pending):
            if len(self.running) >= self.max_active:
                return
            idle = [h for h in self.handles.get(req.key, []) if not h.busy]
            if idle:
                self.pending.remove(req)
                self._start(req, idle[0])
        wanted = {r.key for r in self.pending}
        now_blocked = set()
        for req in list(self.pending):
            if len(self.running) >= self.max_active:
                break
            if req.key in now_blocked:
                continue
            hs = self.handles.get(req.key, [])
            idle = [h for h in hs if not h.busy]
            if idle:
                self.pending.remove(req)
                self._start(req, idle[0])
                continue
            in_flight = sum(1 for k, _ in self.setups.values() if k == req.key)
            if len(hs) + in_flight >= self.handles_per_key or in_flight > 0:
                now_blocked.add(req.key)
                continue
            nbytes = self._nbytes(req)
            if nbytes > self.budget:
                self.pending.remove(req)
                req.error = ServeError(f"request needs {nbytes} bytes, more than the whole budget")
                self.rejected.append(req)
                continue
            if not self._evict_for(nbytes, req.key, wanted):
                now_blocked.add(req.key)
                continue
            self._charge(nbytes)
            fut = self._pool.submit(self._make, req.problem)
            self.setups[fut] = (req.key, nbytes)
            now_blocked.add(req.key)

    def _retire(self):
        for slot, (req, h) in list(self.running.items()):
            done, info, code = self.batch.poll(slot)
            if not done:
                continue
            req.done = time.perf_counter()
            req.info = info
            req.code = code
            if self.keep_results:
                req.result = self.batch.result(slot).clone()
            self.batch.remove(slot)
            del self.running[slot]
            h.busy = False
            h.last_used = req.done
            self.finished.append(req)

    def pump(self):
        """One scheduler round: collect setups, admit, step the batch, retire."""
        self._collect_setups()
        self._admit()
        if self.running:
            self.batch.step()
            self.steps += 1
            self._retire()
            return True
        return False

    def run(self, arrivals=None, timeout=600.0, progress=None, progress_every=5.0):
        """Drive the server until every request (and every timed arrival
        ``(t_offset, Request)``, sorted by offset) is finished or rejected.
        ``progress(server, elapsed_s)``, if given, is called every
        ``progress_every`` seconds."""
        t0 = time.perf_counter()
        t_report = t0
        arrivals = collections.deque(arrivals or [])
        while True:
            if progress is not None and time.perf_counter() - t_report >= progress_every:
                t_report = time.perf_counter()
                progress(self, t_report - t0)
            now = time.perf_counter()
            while arrivals and t0 + arrivals[0][0] <= now:
                off, req = arrivals.popleft()
                req.arrival = t0 + off
                self.submit(req)
            busy = self.pump()
            if not arrivals and self.idle():
                break
            if not busy:
                if self.setups:
                    cf.wait(list(self.setups), timeout=0.002, return_when=cf.FIRST_COMPLETED)
                elif arrivals:
                    time.sleep(max(0.0, min(0.002, t0 + arrivals[0][0] - time.perf_counter())))
            if time.perf_counter() - t0 > timeout:
                raise ServeError("serving run exceeded its timeout")
        return time.perf_counter() - t0

    def stats(self, makespan):
        lat = np.array([r.latency for r in self.finished]) if self.finished else np.zeros(1)
        dofs = sum(r.n for r in self.finished)
        return {"requests": len(self.finished), "rejected": len(self.rejected),
                "failed": sum(1 for r in self.finished if r.code != 0),
                "makespan_s": makespan, "dofs_per_s": dofs / makespan if makespan > 0 else 0.0,
                "requests_per_s": len(self.finished) / makespan if makespan > 0 else 0.0,
                "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                               "p99": 1e3 * float(np.percentile(lat, 99)),
                               "max": 1e3 * float(lat.max())},
                "steps": self.steps, "peak_hbm_bytes": self.peak_used, "budget_bytes": self.budget,
                "evictions": sum(1 for e in self.events if e[1] == "evict")}


# ---------------------------------------------------------------- workload
def request_mix(n_requests, seed=5, n_families=12, **family_kw):
    """Seeded serving workload: ``n_families`` problem families (see
    ``workloads.serving_families``) and ``n_requests`` requests drawn from them."""
    from . import workloads as W
    fams = W.serving_families(n_families, seed=seed, **family_kw)
    return fams, requests_for(fams, n_requests, seed + 1)


def requests_for(fams, n_requests, seed):
    """Requests drawn uniformly from the families, each with its own seeded
    U[-1,1] right-hand side."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    keys = [problem_key(f) for f in fams]
    reqs = []
    for _ in range(n_requests):
        j = int(rng.integers(0, len(fams)))
        s = int(rng.integers(0, 2 ** 31))
        reqs.append(Request(fams[j], (lambda n, s=s: W.random_rhs(n, s)), key=keys[j]))
    return reqs


def poisson_offsets(n, rate, seed):
    """Arrival times of a Poisson process of the given rate (requests/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
