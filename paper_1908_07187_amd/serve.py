"""Continuous-batching circuit server over the C ABI.

Jobs (a circuit and a dtype) arrive over time.  The loop, run on the host:

* admits arrived jobs in arrival order while their device footprint fits
  the HBM budget (``footprint``: the state of 2^n x 8 or 16 bytes; on a
  stream slot also the simulator's fixed buffers and, for circuits with
  permutation gates, a second state-sized buffer) -- a job that can never fit
  is refused with an error, never allowed to exhaust device memory;
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
  device;
* polls completion events and, for each finished job, reads its cbits and a
  digest (norm; for small jobs the whole state) back to the host, frees its
  memory and records its latency (arrival -> result on the host).  A
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
from .qk import Batch, QKError, Sim
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
    def __init__(self, hbm_budget: Optional[int] = None, slots: int = 8,
                 fusion: Optional[Dict[str, int]] = None, keep_states: Sequence[int] = (),
                 small_max: Optional[Dict[str, int]] = None, poll_sleep: float = 20e-6,
                 autotuned: bool = False, mid_max: Optional[Dict[str, int]] = None, stages: bool = False):
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
        # batch pools: small jobs ("c128", "c64") and mid-size jobs ("mid-c128", "mid-c64")
        pools = ("c128", "c64", "mid-c128", "mid-c64")
        bstreams = {p: [torch.cuda.Stream(), torch.cuda.Stream()] for p in pools}
        bpool = {p: [Batch(p.split("-")[-1], stream=s) for s in bstreams[p]] for p in pools}
        bfree = {p: deque(range(2)) for p in pools}
        pending: deque = deque()
        inflight_stream = []   # (slot, sim, event, job index)
        inflight_batch = []    # (dtype, pool index, event, [(job index, batch job id)])
        used = 0
        nxt = 0
        finished = 0
        nbatches = 0
        max_conc = 0
        slept = 0.0            # host time spent waiting (nothing to admit or no room)
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        reported = 0
        while finished < N:
            if progress_every and finished - reported >= progress_every:
                reported = finished - finished % progress_every
                print(f"[serve] {finished}/{N} jobs done at {now():.1f} s", file=sys.stderr, flush=True)
            t = now()
            while nxt < N and arrivals[nxt] <= t:
                res[nxt].arrival = arrivals[nxt]
                pending.append(nxt)
                nxt += 1

            # ---- completions
            still = []
            for slot, sim, ev, j in inflight_stream:
                if ev.query():
                    r = res[j]
                    try:
                        r.cbits = sim.read_cbits()
                        r.norm2 = sim.norm2()
                        if j in self.keep_states:
                            r.state = sim.state()
                    except QKError as e:
                        r.path, r.error = "failed", str(e)
                    r.done = now()
                    sim.close()
                    used -= footprint(r.n, r.dtype, jobs[j][1])
                    free_slots.append(slot)
                    finished += 1
                else:
                    still.append((slot, sim, ev, j))
            inflight_stream = still
            still = []
            for dt, pi, ev, members in inflight_batch:
                if ev.query():
                    b = bpool[dt][pi]
                    for j, bj in members:
                        r = res[j]
                        if r.n <= self.small_max[r.dtype] or j in self.keep_states:
                            r.state = b.state(bj)
                            r.norm2 = float(np.vdot(r.state, r.state).real)
                        r.cbits = b.cbits(bj)
                        r.done = now()
                        used -= footprint(r.n, r.dtype, batched=True)
                        finished += 1
                    b.clear()
                    bfree[dt].append(pi)
                else:
                    still.append((dt, pi, ev, members))
            inflight_batch = still

            # ---- admission (arrival order; a job that does not fit yet waits, later small ones may pass)
            small: Dict[str, List[int]] = {p: [] for p in pools}
            keep = deque()
            while pending:
                j = pending.popleft()
                _, circ, dt = jobs[j]
                r = res[j]
                small_job = r.n <= self.mid_max[dt] and recs[j] is not None
                pool = dt if r.n <= self.small_max[dt] else "mid-" + dt
                fp = footprint(r.n, dt, circ, batched=small_job)
                if fp > self.budget:
                    r.path, r.error = "refused", f"state of {r.n} qubits ({fp} B) exceeds the HBM budget"
                    r.done = now()
                    finished += 1
                    continue
                if used + fp > self.budget:
                    keep.append(j)
                    continue
                if small_job:
                    if bfree[pool]:
                        small[pool].append(j)
                        used += fp
                        r.admitted = now()
                    else:
                        keep.append(j)
                    continue
                if not free_slots:
                    keep.append(j)
                    continue
                slot = free_slots.popleft()
                used += fp
                r.admitted = now()
                r.path = "stream"
                sim = None
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
                    sim.flush()
                    ev = torch.cuda.Event()
                    ev.record(streams[slot])
                    inflight_stream.append((slot, sim, ev, j))
                except QKError as e:
                    if sim is not None:
                        sim.close()
                    r.path, r.error = "failed", str(e)
                    r.done = now()
                    used -= fp
                    free_slots.append(slot)
                    finished += 1
            pending = keep
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
                        used -= footprint(r.n, r.dtype, batched=True)
                        finished += 1
                if members:
                    b.run()
                    ev = torch.cuda.Event()
                    ev.record(bstreams[dt][pi])
                    inflight_batch.append((dt, pi, ev, members))
                    nbatches += 1
                else:
                    bfree[dt].append(pi)
            max_conc = max(max_conc, len(inflight_stream))
            idle = ((finished < N and not pending and (nxt >= N or arrivals[nxt] > now()))
                    or (finished < N and pending and not (free_slots or any(bfree[d] for d in bfree))))
            if idle:
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
                           extra={"host_wait_s": slept, "host_busy_frac": 1.0 - slept / wall if wall > 0 else None})
