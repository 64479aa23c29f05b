"""Continuous-batching circuit server over the C ABI.

Jobs (a circuit and a dtype) arrive over time.  The loop, run on the host:

* queues each arrived job by its route (a batch pool by dtype and size, or
  a stream slot of its own; worked out once per job) and admits each queue in
  arrival order while the head's device footprint fits the HBM budget
  (``footprint``: the state of 2^n x 8 or 16 bytes; on a stream slot also
  the simulator's fixed buffers and, for circuits with permutation gates, a
  second state-sized buffer) -- a job that can never fit is refused with an
  error, never allowed to exhaust device memory; a head that does not fit
  yet waits, and other queues may pass it (scanning one arrival-ordered list
  of every waiting job on each turn of the loop made the closed loop
  quadratic in the queue length);
* takes each request as qk_op records prepared before it arrives (the form a
  client would submit), so a job on a stream slot is enqueued with one C call
  (qk_apply_ops) instead of one call per operation;
* packs admitted small jobs (<= 13 qubits complex128, <= 14 complex64) into
  one persistent batch launch per dtype (``qk_batch_run``), up to two batch
  launches in flight per dtype, so jobs that arrive while a batch runs go into
  the next one;
* optionally (``mid_max``) packs mid-size jobs, above that and up to mid_max
  qubits, into batch launches of their own (the batch kernel runs them by
  stages through LDS, one workgroup per job), kept apart from the small jobs'
  batches so a long mid-size batch never holds back small results;
* gives every admitted large job its own stream slot and enqueues its whole
  circuit there (fused into matrix-core blocks as configured, or as the
  autotuner chose for that qubit count and dtype, or with ``stages`` in the
  LDS-tile mode); slots run concurrently, so their sweeps overlap on the
  device; with ``short_first`` > 0 a free slot takes the oldest waiting job
  of at most that many qubits before any larger one (shorter waits for
  short jobs up to about 0.8 of capacity, a longer tail for long jobs near
  saturation; off by default);
* polls completion events and, for each finished job, takes its cbits and a
  digest (norm; for small jobs the whole state) on the host, frees its memory
  and records its latency (arrival -> result on the host).  A stream-slot job
  enqueues its digest right after its circuit (qk_norm2_async,
  qk_read_cbits_async into pinned host memory), and a batch the copy of all
  its states and cbits right after its launch (qk_batch_read_async), so
  reading a result never waits on the device: copies enqueued only once a
  job had finished queued behind other streams' sweeps (about 5 ms per small
  job).  A
  mid-size batched job's state is read back only when asked for
  (``keep_states``), and so is its norm.

States stay resident in HBM for the whole circuit; nothing but the result
crosses to the host.  A job's result does not depend on the other jobs in
flight: every kernel is deterministic and every reduction runs in a fixed
order that depends only on the job.
"""
from __future__ import annotations

import gc
import sys
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import autotune as _autotune
from . import batch as _batch
from .qk import Batch, QKError, Sim, norm2_from_partials
from .runner import Program

SMALL_MAX = {"c128": 13, "c64": 14}
AMP_BYTES = {"c128": 16, "c64": 8}


@dataclass
class JobResult:
    index: int
    n: int
    dtype: str
    path: str = ""                 # 'batch' | 'stream' | 'refused' | 'failed'
    arrival: float = 0.0           # seconds since the server started
    admitted: float = 0.0
    done: float = 0.0
    cbits: Optional[np.ndarray] = None
    norm2: float = float("nan")
    state: Optional[np.ndarray] = None
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeReport:
    results: List[JobResult]
    wall_s: float
    completed: int
    refused: int
    failed: int
    circuits_per_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    batches: int
    max_concurrent_streams: int
    extra: Dict = field(default_factory=dict)


# Device memory a simulator holds beside its state: the constant arena chunk
# of fused block matrices (32 MiB, allocated on first use) and the
# measurement buffers, cbits and diagonal-run tables (under 1 MiB).
SIM_OVERHEAD = (32 << 20) + (1 << 20)
PERM_KINDS = ("table", "affine", "modmul")


def footprint(n: int, dtype: str, circuit=None, batched: bool = False) -> int:
    """Device bytes a job holds while admitted.  A batched job holds its state
    inside the batch buffers; a job on its own stream slot holds its state,
    a second state-sized buffer if it applies permutation gates (they gather
    into it), and the simulator's fixed buffers."""
    state = (1 << n) * AMP_BYTES[dtype]
    if batched:
        return state
    perms = circuit is not None and any(g.get("kind") in PERM_KINDS for g in circuit.user_gates.values())
    return state * (2 if perms else 1) + SIM_OVERHEAD


class Server:
    def __init__(self, hbm_budget: Optional[int] = None, slots: int = 4,
                 fusion: Optional[Dict[str, int]] = None, keep_states: Sequence[int] = (),
                 small_max: Optional[Dict[str, int]] = None, poll_sleep: float = 20e-6,
                 autotuned: bool = False, mid_max: Optional[Dict[str, int]] = None, stages: bool = False,
                 short_first: int = 0):
        import torch
        self.torch = torch
        if hbm_budget is None:
            free, total = torch.cuda.mem_get_info()
            hbm_budget = int(0.85 * free)
        self.budget = int(hbm_budget)
        self.slots = slots
        self.fusion = {"c128": 0, "c64": 5} if fusion is None else dict(fusion)
        self.keep_states = set(keep_states)
        self.small_max = dict(SMALL_MAX if small_max is None else small_max)
        self.mid_max = dict(self.small_max if mid_max is None else mid_max)
        # stream-slot jobs in the LDS-tile mode (gates grouped into stages, no
        # block matrices to compose) instead of fused blocks
        self.stages = stages
        # stream-slot jobs of at most this many qubits are admitted before
        # larger ones (each class in arrival order); 0: one arrival-order queue
        self.short_first = short_first
        self.poll_sleep = poll_sleep
        # large jobs take the autotuner's fusion width and tile shape for their size
        self.tuning_cache = _autotune.load_cache() if autotuned else None
        self.autotuned = bool(self.tuning_cache)

    # ------------------------------------------------------------------
    def serve(self, jobs: Sequence[Tuple[float, object, str]], realtime: bool = True,
              progress_every: int = 0) -> ServeReport:
        """Run ``jobs`` = [(arrival_s, circuit, dtype)] (sorted by arrival).
        realtime=False makes every job arrive at t = 0 (closed-loop saturation).
        progress_every > 0 prints a line to stderr each time that many more
        jobs have finished.

        While the loop runs, the objects that exist when it starts (the queued
        circuits: millions of op objects for a long stream) are frozen out of
        Python's cyclic garbage collector.  Each full collection would
        otherwise traverse all of them, pausing the host loop for 0.4-0.5 s
        about every 10 s of a 3000-job stream, and those pauses set the 99th
        percentile latency."""
        gc.collect()
        gc.freeze()
        try:
            return self._serve(jobs, realtime, progress_every)
        finally:
            gc.unfreeze()

    @staticmethod
    def _records(circ):
        """A request as the loop receives it: qk_op records (one C call per job)
        when the circuit has builtin gates only and starts from |0...0>, else
        None (the circuit is then issued op by op)."""
        if circ.init_state is not None or circ.user_gates:
            return None
        try:
            return _batch.op_array(circ)
        except ValueError:
            return None

    def _serve(self, jobs, realtime, progress_every) -> ServeReport:
        torch = self.torch
        N = len(jobs)
        res = [JobResult(i, c.n_qubits, dt) for i, (_, c, dt) in enumerate(jobs)]
        recs = [self._records(c) for _, c, _ in jobs]
        arrivals = [a if realtime else 0.0 for a, _, _ in jobs]
        streams = [torch.cuda.Stream() for _ in range(self.slots)]
        free_slots = deque(range(self.slots))
        # per slot, pinned host memory the job's digest (norm partial sums and
        # cbits) is copied into right after its circuit, so that a finished
        # job is read without waiting on the device
        norm_host = [torch.empty(2048, dtype=torch.float64, pin_memory=True) for _ in range(self.slots)]
        cbit_host = [torch.empty(256, dtype=torch.uint8, pin_memory=True) for _ in range(self.slots)]
        # batch pools: small jobs ("c128", "c64") and mid-size jobs ("mid-c128", "mid-c64")
        pools = ("c128", "c64", "mid-c128", "mid-c64")
        bstreams = {p: [torch.cuda.Stream(), torch.cuda.Stream()] for p in pools}
        bpool = {p: [Batch(p.split("-")[-1], stream=s) for s in bstreams[p]] for p in pools}
        bfree = {p: deque(range(2)) for p in pools}
        # per batch, pinned host memory its results (every state and cbit) are
        # copied into right after its launch (grown on demand)
        bhost = {p: [[None, None], [None, None]] for p in pools}
        # each job's route, worked out once: its queue (a batch pool, or
        # "stream" for a slot of its own) and its device footprint
        route = []
        for j, (_, circ, dt) in enumerate(jobs):
            batched = res[j].n <= self.mid_max[dt] and recs[j] is not None
            q = (dt if res[j].n <= self.small_max[dt] else "mid-" + dt) if batched else \
                ("stream-short" if res[j].n <= self.short_first else "stream")
            route.append((q, footprint(res[j].n, dt, circ, batched=batched)))
        # arrived, not yet admitted, in arrival order
        waiting = {q: deque() for q in pools + ("stream-short", "stream")}
        inflight_stream = []   # (slot, sim, event, job index, norm partial sums)
        inflight_batch = []    # (dtype, pool index, event, [(job index, batch job id)])
        used = 0
        nxt = 0
        finished = 0
        nbatches = 0
        max_conc = 0
        slept = 0.0            # host time spent waiting (nothing to admit or no room)
        spent = {"stream_enqueue": 0.0, "batch_enqueue": 0.0, "stream_results": 0.0, "batch_results": 0.0,
                 "event_query": 0.0, "stream_close": 0.0}
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        reported = 0
        while finished < N:
            if progress_every and finished - reported >= progress_every:
                reported = finished - finished % progress_every
                print(f"[serve] {finished}/{N} jobs done at {now():.1f} s", file=sys.stderr, flush=True)
            progress = False
            t = now()
            while nxt < N and arrivals[nxt] <= t:
                r = res[nxt]
                r.arrival = arrivals[nxt]
                q, fp = route[nxt]
                if fp > self.budget:
                    r.path, r.error = "refused", f"state of {r.n} qubits ({fp} B) exceeds the HBM budget"
                    r.done = now()
                    finished += 1
                else:
                    waiting[q].append(nxt)
                nxt += 1
                progress = True

            # ---- completions
            still = []
            tq = time.perf_counter()
            for slot, sim, ev, j, nb in inflight_stream:
                tq2 = time.perf_counter()
                done = ev.query()
                spent["event_query"] += time.perf_counter() - tq2
                if done:
                    r = res[j]
                    try:
                        nc = jobs[j][1].n_cbits
                        if nc <= 256:
                            r.cbits = cbit_host[slot][:nc].numpy().copy()
                        else:
                            r.cbits = sim.read_cbits()
                        r.norm2 = norm2_from_partials(norm_host[slot].numpy(), nb)
                        if j in self.keep_states:
                            r.state = sim.state()
                    except QKError as e:
                        r.path, r.error = "failed", str(e)
                    r.done = now()
                    tq2 = time.perf_counter()
                    sim.close()
                    spent["stream_close"] += time.perf_counter() - tq2
                    used -= route[j][1]
                    free_slots.append(slot)
                    finished += 1
                    progress = True
                else:
                    still.append((slot, sim, ev, j, nb))
            inflight_stream = still
            spent["stream_results"] += time.perf_counter() - tq
            still = []
            tq = time.perf_counter()
            for dt, pi, ev, members in inflight_batch:
                if ev.query():
                    b = bpool[dt][pi]
                    hs, hc = bhost[dt][pi]
                    for j, bj in members:
                        r = res[j]
                        so, sb, co = b.layout(bj)
                        if r.n <= self.small_max[r.dtype] or j in self.keep_states:
                            r.state = hs[so:so + sb].numpy().view(b.np_dtype).copy()
                            r.norm2 = float(np.vdot(r.state, r.state).real)
                        r.cbits = hc[co:co + jobs[j][1].n_cbits].numpy().copy()
                        r.done = now()
                        used -= route[j][1]
                        finished += 1
                    b.clear()
                    progress = True
                    bfree[dt].append(pi)
                else:
                    still.append((dt, pi, ev, members))
            inflight_batch = still
            spent["batch_results"] += time.perf_counter() - tq

            # ---- admission: each queue in arrival order; a job whose footprint
            # does not fit yet waits at the head of its queue (jobs of other
            # queues may pass it).  Batch pools take every waiting job that
            # fits when one of their batches is free.
            small: Dict[str, List[int]] = {p: [] for p in pools}
            for p in pools:
                wq = waiting[p]
                while bfree[p] and wq and used + route[wq[0]][1] <= self.budget:
                    j = wq.popleft()
                    small[p].append(j)
                    used += route[j][1]
                    res[j].admitted = now()
            while free_slots:
                # the short-job queue first, then the others
                wq = None
                for qn in ("stream-short", "stream"):
                    cand = waiting[qn]
                    if cand and used + route[cand[0]][1] <= self.budget:
                        wq = cand
                        break
                if wq is None:
                    break
                j = wq.popleft()
                _, circ, dt = jobs[j]
                r = res[j]
                fp = route[j][1]
                slot = free_slots.popleft()
                used += fp
                r.admitted = now()
                r.path = "stream"
                progress = True
                sim = None
                tq = time.perf_counter()
                try:
                    sim = Sim(dt, stream=streams[slot])
                    if self.stages:
                        sim.set_tuning("stages", 1)
                    elif self.autotuned:
                        _autotune.apply(sim, r.n, dt, self.tuning_cache)
                    elif self.fusion.get(dt, 0):
                        sim.set_fusion(self.fusion[dt])
                    if recs[j] is not None:
                        sim.add_qubits(r.n)
                        if circ.n_cbits:
                            sim.add_cbits(circ.n_cbits)
                        sim.apply_ops(*recs[j])
                    else:
                        Program(circ).run(sim)
                    nb = sim.norm2_async(norm_host[slot].data_ptr(), 2048)
                    if 0 < circ.n_cbits <= 256:
                        sim.read_cbits_async(cbit_host[slot].data_ptr(), circ.n_cbits)
                    ev = torch.cuda.Event()
                    ev.record(streams[slot])
                    inflight_stream.append((slot, sim, ev, j, nb))
                    spent["stream_enqueue"] += time.perf_counter() - tq
                except QKError as e:
                    if sim is not None:
                        sim.close()
                    r.path, r.error = "failed", str(e)
                    r.done = now()
                    used -= fp
                    free_slots.append(slot)
                    finished += 1
            tq = time.perf_counter()
            for dt in pools:
                if not small[dt]:
                    continue
                pi = bfree[dt].popleft()
                b = bpool[dt][pi]
                members = []
                for j in small[dt]:
                    r = res[j]
                    r.path = "batch"
                    try:
                        circ = jobs[j][1]
                        members.append((j, b.add(circ.n_qubits, circ.n_cbits, recs[j][0], recs[j][1])))
                    except (QKError, ValueError) as e:
                        r.path, r.error = "failed", str(e)
                        r.done = now()
                        used -= route[j][1]
                        finished += 1
                if members:
                    b.run()
                    nbytes, ncb = b.sizes()
                    hs, hc = bhost[dt][pi]
                    if hs is None or hs.numel() < nbytes:
                        hs = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, pin_memory=True)
                    if hc is None or hc.numel() < max(ncb, 1):
                        hc = torch.empty(max(ncb, 4096), dtype=torch.uint8, pin_memory=True)
                    bhost[dt][pi] = [hs, hc]
                    b.read_async(hs.data_ptr(), hs.numel(), hc.data_ptr(), hc.numel())
                    ev = torch.cuda.Event()
                    ev.record(bstreams[dt][pi])
                    inflight_batch.append((dt, pi, ev, members))
                    nbatches += 1
                    progress = True
                else:
                    bfree[dt].append(pi)
            spent["batch_enqueue"] += time.perf_counter() - tq
            max_conc = max(max_conc, len(inflight_stream))
            # nothing arrived, finished or started: wait a little before polling again
            if not progress and finished < N:
                ts = time.perf_counter()
                time.sleep(self.poll_sleep)
                slept += time.perf_counter() - ts

        wall = now()
        for dt in bpool:
            for b in bpool[dt]:
                b.close()
        ok = [r for r in res if r.path in ("batch", "stream")]
        lat = np.array([r.latency for r in ok]) * 1e3 if ok else np.array([0.0])
        span = (max(r.done for r in ok) - min(r.arrival for r in ok)) if ok else wall
        return ServeReport(results=res, wall_s=wall, completed=len(ok),
                           refused=sum(r.path == "refused" for r in res),
                           failed=sum(r.path == "failed" for r in res),
                           circuits_per_s=len(ok) / span if span > 0 else float("nan"),
                           p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                           mean_ms=float(lat.mean()), batches=nbatches, max_concurrent_streams=max_conc,
                           extra={"host_wait_s": slept, "host_busy_frac": 1.0 - slept / wall if wall > 0 else None,
                                  "host_s": spent})
