"""Continuous-batching server for encrypted bag-of-words inference.

Requests (an encrypted count vector, already resident on the device, plus
the word count w) arrive over time for one of several parameter sets.  Each
parameter set has its own context, HIP stream, resident evaluation keys and
plaintext model (Sec. 4.1: v H, x 1/w, h O).  The scheduler:
  * queues arrivals per parameter set (FIFO);
  * whenever a parameter set's stream has no batch in flight, admits the
    oldest waiting requests of that set as one batch, as many as fit in the
    HBM budget and the batch cap.  A set's device footprint beyond its keys
    is the larger of its in-flight batch's working set and the scratch its
    context keeps allocated from earlier batches (the library's workspace
    only grows), so the sum over sets of that footprint stays within the
    budget;
  * launches the batch asynchronously and polls completion, so batches of
    different parameter sets overlap on the device and requests that arrive
    meanwhile join the next batch (continuous batching);
  * rejects requests whose working set alone exceeds the budget.
Results do not depend on the batch a request lands in: every batched kernel
treats its ciphertexts independently.

The executor is pluggable: GpuExecutor runs libpft; tests drive the
scheduler with a simulated executor and clock on the CPU.
"""

import time
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    pset: str           # parameter-set name
    arrival: float      # seconds from the start of the trace
    doc: int            # index of the pre-encrypted document in its pool
    words: int          # w, sent in plaintext (Sec. 4.1)
    admitted: float = None
    done: float = None
    rejected: bool = False
    result: object = None


@dataclass
class PsetPolicy:
    bytes_per_request: int
    max_batch: int


@dataclass
class Stats:
    latencies: list = field(default_factory=list)
    makespan: float = 0.0
    completed: int = 0
    rejected: int = 0
    batches: int = 0

    def percentile(self, p):
        xs = sorted(self.latencies)
        if not xs:
            return None
        k = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
        return xs[k]

    def summary(self):
        return {
            "completed": self.completed,
            "rejected": self.rejected,
            "batches": self.batches,
            "req_per_s": self.completed / self.makespan if self.makespan > 0 else None,
            "p50_ms": None if not self.latencies else 1000.0 * self.percentile(50),
            "p99_ms": None if not self.latencies else 1000.0 * self.percentile(99),
            "mean_batch": self.completed / self.batches if self.batches else None,
        }


class RealClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def sleep_until(self, t):
        dt = t - self.now()
        if dt > 0:
            time.sleep(min(dt, 0.0005))


class Scheduler:
    def __init__(self, executor, policies, budget_bytes, clock=None, continuous=True):
        """policies: {pset: PsetPolicy}.  continuous=False gives the plain
        per-op server: one request at a time, in arrival order, no overlap.
        The executor may provide retained(pset): device bytes the set keeps
        allocated between batches (0 if absent)."""
        self.ex = executor
        self.policies = policies
        self.budget = budget_bytes
        self.clock = clock or RealClock()
        self.continuous = continuous
        self.used = 0
        self.inflight_bytes = {}

    def _retained(self, p):
        f = getattr(self.ex, "retained", None)
        return f(p) if f else 0

    def _footprint(self, skip=None):
        """Device bytes beyond keys over all sets (except `skip`): per set the
        larger of its in-flight working set and its retained scratch."""
        return sum(max(self._retained(p), self.inflight_bytes.get(p, 0)) for p in self.policies if p != skip)

    def run(self, trace):
        """Serve every request of `trace` (sorted by arrival); fills in
        admitted/done/rejected and returns Stats."""
        stats = Stats()
        pending = list(trace)
        pending.sort(key=lambda r: r.arrival)
        queues = {p: [] for p in self.policies}
        inflight = {}      # pset -> (handle, requests, bytes)
        order = []         # FIFO of waiting requests across sets (per-op server)
        i = 0
        while i < len(pending) or any(queues.values()) or inflight:
            now = self.clock.now()
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                i += 1
                if self.policies[r.pset].bytes_per_request > self.budget:
                    r.rejected = True
                    stats.rejected += 1
                    continue
                queues[r.pset].append(r)
                order.append(r)
            # completions
            for p in list(inflight):
                h, reqs, nbytes = inflight[p]
                if self.ex.poll(h):
                    t = self.clock.now()
                    for r, res in zip(reqs, self.ex.results(h)):
                        r.done = t
                        r.result = res
                        stats.latencies.append(r.done - r.arrival)
                        stats.completed += 1
                    self.used -= nbytes
                    self.inflight_bytes.pop(p, None)
                    del inflight[p]
            # admissions
            if self.continuous:
                for p in sorted(queues, key=lambda q: queues[q][0].arrival if queues[q] else float("inf")):
                    if p in inflight or not queues[p]:
                        continue
                    pol = self.policies[p]
                    # the set's scratch already allocated covers that much of a batch
                    room = self.budget - self._footprint(skip=p)
                    fit = room // pol.bytes_per_request
                    n = min(len(queues[p]), pol.max_batch, fit)
                    if n <= 0:
                        continue
                    batch, queues[p] = queues[p][:n], queues[p][n:]
                    self._launch(p, batch, inflight, stats)
            elif not inflight and order:
                r = order.pop(0)
                queues[r.pset].remove(r)
                self._launch(r.pset, [r], inflight, stats)
            if i < len(pending) and not inflight and not any(queues.values()):
                self.clock.sleep_until(pending[i].arrival)
            else:
                self.clock.sleep_until(self.clock.now() + 0.0002)
        stats.makespan = self.clock.now() - (trace[0].arrival if trace else 0.0)
        return stats

    def _launch(self, p, batch, inflight, stats):
        nbytes = self.policies[p].bytes_per_request * len(batch)
        self.used += nbytes
        self.inflight_bytes[p] = nbytes
        t = self.clock.now()
        for r in batch:
            r.admitted = t
        inflight[p] = (self.ex.submit(p, batch), batch, nbytes)
        stats.batches += 1


def poisson_trace(seed, n_requests, rate, mix, pools, word_counts):
    """Arrivals of a Poisson process of `rate` requests/s; each request picks
    a parameter set with the weights of `mix` ({pset: weight}) and a document
    of that set's pool (pools: {pset: pool size}); word_counts: {pset: [w]}."""
    import numpy as np
    g = np.random.default_rng(seed)
    names = sorted(mix)
    w = np.array([mix[n] for n in names], dtype=np.float64)
    w /= w.sum()
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += g.exponential(1.0 / rate)
        p = names[int(g.choice(len(names), p=w))]
        doc = int(g.integers(0, pools[p]))
        out.append(Request(rid, p, t, doc, int(word_counts[p][doc])))
    return out


class GpuExecutor:
    """Runs batches with libpft: one context (and HIP stream) per parameter
    set, inputs from a device-resident pool of encrypted documents."""

    def __init__(self, sets):
        """sets: {pset: (ctx, model, pool)} with pool[doc] = list of input
        ciphertexts of that document."""
        import torch
        self.torch = torch
        self.sets = sets
        self.handles = {}
        self.next = 0

    def submit(self, p, batch):
        from .inference import encrypted_inference
        ctx, model, pool = self.sets[p]
        out = encrypted_inference(ctx, model, [pool[r.doc] for r in batch], [r.words for r in batch])
        ev = self.torch.cuda.Event()
        ev.record(ctx.stream)
        h = self.next
        self.next += 1
        self.handles[h] = (ev, out)
        return h

    def poll(self, h):
        return self.handles[h][0].query()

    def results(self, h):
        return self.handles.pop(h)[1]

    def retained(self, p):
        """Scratch bytes (workspaces, buffers of composite operations) the
        set's context keeps allocated between batches."""
        return int(self.sets[p][0].memory()["scratch"])


class SimExecutor:
    """Simulated device for CPU tests: a batch of n requests of set p takes
    cost(p, n) seconds of simulated time; sets run concurrently."""

    def __init__(self, clock, cost, retain=None):
        """retain(p, n): scratch a batch of n requests of set p leaves
        allocated (the set keeps the largest so far); None: nothing."""
        self.clock = clock
        self.cost = cost
        self.retain = retain
        self.kept = {}
        self.jobs = {}
        self.next = 0
        self.log = []

    def submit(self, p, batch):
        h = self.next
        self.next += 1
        self.jobs[h] = (self.clock.now() + self.cost(p, len(batch)), [("result", r.rid) for r in batch])
        self.log.append((self.clock.now(), p, [r.rid for r in batch]))
        if self.retain:
            self.kept[p] = max(self.kept.get(p, 0), self.retain(p, len(batch)))
        return h

    def retained(self, p):
        return self.kept.get(p, 0)

    def poll(self, h):
        return self.clock.now() >= self.jobs[h][0]

    def results(self, h):
        return self.jobs.pop(h)[1]


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


def request_bytes(params, n_in, b, level):
    """Device bytes a request of this parameter set holds while in flight:
    its inputs, the PtMatVec buffers (baby rotations + three accumulators)
    and one key-switching workspace."""
    n = params.n
    ct = 2 * level * n * 8
    K, alpha = params.K, params.alpha
    beta = -(-level // alpha)
    rows = level + K
    ks = (2 * level + level + beta * rows + 2 * rows + 2 * level) * n * 8
    return (n_in + n_in * b + 3 + 4) * ct + ks


def key_bytes(params):
    """Device bytes of one switching key: [dnum][2][L+K][N] words."""
    return params.dnum * 2 * (params.L + params.K) * params.n * 8


def build_sets(specs, H, O, pool_size, level, draws, key_seed=77, doc_seed=78, key_budget_bytes=None):
    """One context (own HIP stream), evaluation keys, plaintext model and a
    pool of encrypted documents per parameter set.
    specs: {name: WorkloadConfig-like}; draws: the seeded input module
    providing key_draws/switch_key_draws/enc_draws/bow_documents.
    key_budget_bytes: device bytes for rotation keys across all sets (None:
    every key resident); a set whose keys exceed its equal share keeps as
    many as fit in device slots and the rest in pinned host memory (the
    rotation-key cache), so it is still admitted.
    Returns (executor sets, policies, word counts, plain counts)."""
    import torch

    from .ckks import Context, Params
    from .inference import BowModel, split_counts

    sets, policies, words, counts_all = {}, {}, {}, {}
    vocab = H.shape[0]
    for name, cfg in specs.items():
        lp = Params.from_config(cfg)
        ctx = Context(lp, 0, stream=torch.cuda.Stream())
        n = lp.n
        kd = draws.key_draws(key_seed, n, lp.q)
        ctx.set_secret(kd.s)
        ctx.gen_public_key(kd.pk_a, kd.pk_e)
        model = BowModel(ctx, H, O, level)
        steps = model.rotation_steps()
        if key_budget_bytes is not None:
            share = key_budget_bytes // len(specs)
            kb = key_bytes(lp)
            if len(steps) * kb > share:
                ctx.set_key_cache(max(1, share // kb))
                ctx.key_cache_plan(model.rotation_order())
        for st in steps:
            a, e = draws.switch_key_draws(key_seed, 5000 + st, n, lp.key_moduli(), lp.dnum)
            ctx.gen_rotation_key(st, a, e)
        counts, w = draws.bow_documents(doc_seed, pool_size, vocab)
        pool = []
        for d in range(pool_size):
            cts = []
            for c, v in enumerate(split_counts(counts[d], model.n_in, model.t)):
                r = draws.enc_draws(doc_seed * 1000 + d * 16 + c, n)
                cts.append(ctx.encrypt(lp.encode(v), level, lp.scale, r.v, r.e0, r.e1))
            pool.append(cts)
        ctx.synchronize()
        sets[name] = (ctx, model, pool)
        policies[name] = PsetPolicy(request_bytes(lp, model.n_in, model.stage1.b, level), 32)
        words[name] = w
        counts_all[name] = counts
    return sets, policies, words, counts_all
