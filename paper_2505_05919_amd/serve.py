"""Continuous-batching job server for CVF Monte Carlo jobs on one GPU.

Jobs (L, T, P, nsteps, algorithm, seed) arrive over time.  The server admits
them in arrival order while their device footprint fits the memory budget and
a slot is free, keeps every admitted lattice resident in HBM, and advances all
resident jobs together in quanta: the Metropolis jobs as one batched launch
per colour phase, the Swendsen-Wang jobs as one batched launch per SW stage
(``cvf_batch_*``) on a second stream, so that the two batches overlap on the
device.  Jobs that finish leave between
quanta and queued jobs take their place, so requests that arrive while others
run are admitted as memory and slots free up.

Every job's result is a pure function of its parameters and seed: identical
alone and in the mix (tested).  An optional policy (policy.AlgoPolicy)
chooses each job's algorithm when it arrives.  All device work goes through
libcvf.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import cvf
from .policy import AlgoPolicy
from .workloads import Job


def footprint(job: Job) -> int:
    """Device bytes a resident job holds: sigma planes plus its workspace."""
    p = cvf.cvf_params_from_si(job.T, job.P, L=job.L, seed=job.seed)
    mask = cvf.CVF_ALGO_METROPOLIS | (cvf.CVF_ALGO_SW if job.algo == "sw" else 0)
    return 4 * job.L * job.L + cvf.cvf_workspace_bytes(p, mask)


@dataclass
class Running:
    job: Job
    chain: cvf.Chain
    done: int = 0
    admitted_at: float = 0.0
    t_ref: float = 0.0          # latency origin: the arrival (realtime) or the release


@dataclass
class Record:
    job: Job
    admitted: float
    completed: float
    obs: dict
    digest: str = ""
    t_ref: float = 0.0

    @property
    def latency(self):
        return self.completed - self.t_ref

    @property
    def queueing(self):
        return self.admitted - self.t_ref


@dataclass
class Server:
    memory_budget: int = 8 << 30        # bytes of HBM the server may keep resident
    max_slots: int = 512                # resident jobs
    quantum: int = 50                   # MC steps per quantum for every resident job
    graph_block: int = 0                # >0: batched sweeps replay a hipGraph of this many
    keep_digest: bool = False
    digest_seeds: frozenset | None = None   # with keep_digest: only these jobs' sigma is hashed (None: all)
    policy: AlgoPolicy | None = None    # algorithm choice at arrival (None: as submitted)
    # quantum membership: "all" advances every resident job (processor
    # sharing); "srpt" advances the resident jobs with the least remaining
    # work first, adding jobs (per algorithm) until a quantum holds at least
    # fill_cells lattice cells, so short jobs finish early while the batch
    # still fills the GPU
    schedule: str = "all"
    fill_cells: int = 1 << 24
    records: list = field(default_factory=list)
    peak_resident_bytes: int = 0
    peak_resident_jobs: int = 0
    quanta: int = 0
    # wall seconds per part of the loop: admission (chain creation), enqueueing
    # the quantum's launches (of which batch rebuilds), waiting for the GPU,
    # retiring finished jobs (of which sigma digests)
    phase_s: dict = field(default_factory=lambda: {"admit": 0.0, "launch": 0.0, "wait": 0.0, "retire": 0.0,
                                                   "rebuild": 0.0, "digest": 0.0})

    def _members(self, runs: list) -> list:
        if self.schedule == "srpt":
            return _srpt(runs, self.fill_cells)
        return runs

    def run(self, jobs: list[Job], realtime: bool = True) -> list[Record]:
        """Serve `jobs` (sorted by arrival).  realtime: arrivals are released
        by the wall clock from the start of the call; otherwise all jobs are
        available at once (arrival times are still used for latencies).

        The loop keeps one quantum in flight: every job's step count advances
        when its quantum is enqueued, so the members of quantum k + 1 are
        known before quantum k ends; the loop enqueues k + 1 (behind k on the
        same streams) and only then waits for k.  Nothing the host does
        between quanta waits for the GPU: chains are created with kernels
        only, batches upload their descriptors from pinned staging, and a
        finishing job's observables (and sigma, when digested) are copied to
        pinned host memory on its stream right after its last quantum, to be
        read once that quantum's event has completed."""
        import ctypes
        import hashlib

        import torch
        stream_b = torch.cuda.current_stream()
        stream_s = torch.cuda.Stream()             # default priority
        pending = list(jobs)
        queue: list[Job] = []
        running: list[Running] = []                # admitted, steps left to enqueue
        used = 0
        batch = None
        batch_members: tuple = ()
        swb = None
        swb_members: tuple = ()
        inflight = None                            # (events, [(run, obs buffer, sigma copy)], batches to close)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0     # noqa: E731
        obs_bytes = ctypes.sizeof(cvf.cvf_obs)

        def collect(runs, st):
            """Enqueue on st, behind the runs' last quantum, the copies their
            retirement reads."""
            out = []
            with torch.cuda.stream(st):
                for r in runs:
                    ob = torch.empty(obs_bytes, dtype=torch.uint8, pin_memory=True)
                    cvf.cvf_observables_async(r.chain.h, ob.data_ptr(), st)
                    sg = None
                    if self.keep_digest and (self.digest_seeds is None or r.job.seed in self.digest_seeds):
                        sg = torch.empty(r.chain.sigma.numel(), dtype=torch.uint8, pin_memory=True)
                        sg.copy_(r.chain.sigma, non_blocking=True)
                    out.append((r, ob, sg))
            return out

        def retire(q):
            events, finishing, stale = q
            tw0 = time.perf_counter()
            for ev in events:
                ev.synchronize()
            tdone = now()
            tw = time.perf_counter()
            self.phase_s["wait"] += tw - tw0
            nonlocal used
            for b in stale:
                b.close()
            for r, ob, sg in finishing:
                o = cvf.cvf_obs.from_buffer_copy(ob.numpy().tobytes()).as_dict()
                tb = time.perf_counter()
                dg = hashlib.sha256(sg.numpy().tobytes()).hexdigest() if sg is not None else ""
                self.phase_s["digest"] += time.perf_counter() - tb
                self.records.append(Record(r.job, r.admitted_at, tdone, o, dg, r.t_ref))
                used -= footprint(r.job)
                r.chain.close()
            self.phase_s["retire"] += time.perf_counter() - tw

        while pending or queue or running or inflight is not None:
            tnow = now()
            tp = time.perf_counter()
            while pending and (not realtime or pending[0].arrival <= tnow):
                job = pending.pop(0)
                queue.append(self.policy.apply(job) if self.policy else job)
            # admission: FIFO, by footprint and slots (jobs a quantum in flight
            # finishes still hold their memory until they are retired)
            held = len(running) + (len(inflight[1]) if inflight is not None else 0)
            while queue and held < self.max_slots:
                fp = footprint(queue[0])
                if used + fp > self.memory_budget and held:
                    break
                job = queue.pop(0)
                p = cvf.cvf_params_from_si(job.T, job.P, L=job.L, seed=job.seed)
                mask = cvf.CVF_ALGO_METROPOLIS | (cvf.CVF_ALGO_SW if job.algo == "sw" else 0)
                st = stream_s if job.algo == "sw" else stream_b
                with torch.cuda.stream(st):
                    ch = cvf.Chain(p, mask, stream=st)
                    ch.set_stop(job.nsteps)            # quanta may overshoot; the chain stops exactly
                running.append(Running(job, ch, 0, now(), job.arrival if realtime else 0.0))
                used += fp
                held += 1
                self.peak_resident_bytes = max(self.peak_resident_bytes, used)
                self.peak_resident_jobs = max(self.peak_resident_jobs, held)
            tq = time.perf_counter()
            self.phase_s["admit"] += tq - tp
            if not running:
                if inflight is not None:
                    retire(inflight)
                    inflight = None
                elif pending:
                    time.sleep(max(0.0, min(pending[0].arrival - now(), 0.002)))
                continue
            met = self._members([r for r in running if r.job.algo == "met"])
            sws = self._members([r for r in running if r.job.algo == "sw"])
            stale, events, finishing = [], [], []
            # one quantum: every member advances by min(quantum, remaining) steps
            if met:
                steps = min(self.quantum, max(r.job.nsteps - r.done for r in met))
                members = tuple(id(r) for r in met)
                if members != batch_members:
                    if batch is not None:
                        stale.append(batch)            # closed once the quantum in flight is done
                    tr = time.perf_counter()
                    batch = cvf.Batch([r.chain for r in met], stream=stream_b, nowait=True)
                    self.phase_s["rebuild"] += time.perf_counter() - tr
                    batch_members = members
                batch.metropolis(steps, graph_block=self.graph_block if steps % max(1, self.graph_block) == 0 else 0)
                for r in met:
                    r.done = min(r.done + steps, r.job.nsteps)
                finishing += collect([r for r in met if r.done >= r.job.nsteps], stream_b)
                events.append(torch.cuda.Event())
                events[-1].record(stream_b)
            if sws:
                n = min(self.quantum, max(r.job.nsteps - r.done for r in sws))
                members = tuple(id(r) for r in sws)
                if members != swb_members:
                    if swb is not None:
                        stale.append(swb)
                    tr = time.perf_counter()
                    swb = cvf.Batch([r.chain for r in sws], stream=stream_s, nowait=True)
                    self.phase_s["rebuild"] += time.perf_counter() - tr
                    swb_members = members
                swb.sw(n)
                for r in sws:
                    r.done = min(r.done + n, r.job.nsteps)
                finishing += collect([r for r in sws if r.done >= r.job.nsteps], stream_s)
                events.append(torch.cuda.Event())
                events[-1].record(stream_s)
            running = [r for r in running if r.done < r.job.nsteps]
            if finishing:
                # a finished job leaves its batch: rebuild at the next quantum
                if any(r.job.algo == "met" for r, _, _ in finishing):
                    batch_members = ()
                if any(r.job.algo == "sw" for r, _, _ in finishing):
                    swb_members = ()
            self.quanta += 1
            self.phase_s["launch"] += time.perf_counter() - tq
            if inflight is not None:
                retire(inflight)
            inflight = (events, finishing, stale)
        for b in (batch, swb):
            if b is not None:
                b.close()
        return self.records


def _remaining_work(r: Running) -> int:
    return (r.job.nsteps - r.done) * r.job.L * r.job.L


def _srpt(runs: list, fill_cells: int) -> list:
    """The runs with the least remaining work, until they hold fill_cells
    cells per step."""
    out, cells = [], 0
    for r in sorted(runs, key=lambda r: (_remaining_work(r), r.job.seed)):
        out.append(r)
        cells += r.job.L * r.job.L
        if cells >= fill_cells:
            break
    return out


def run_alone(job: Job) -> tuple[dict, str, float]:
    """One job with plain single-chain launches; returns (observables,
    sigma digest, service seconds)."""
    import hashlib

    import torch
    p = cvf.cvf_params_from_si(job.T, job.P, L=job.L, seed=job.seed)
    mask = cvf.CVF_ALGO_METROPOLIS | (cvf.CVF_ALGO_SW if job.algo == "sw" else 0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ch = cvf.Chain(p, mask)
    (ch.metropolis if job.algo == "met" else ch.sw)(job.nsteps)
    o = ch.obs()
    dt = time.perf_counter() - t
    dg = hashlib.sha256(ch.sigma.cpu().numpy().tobytes()).hexdigest()
    ch.close()
    return o, dg, dt


def fcfs_latencies(jobs: list[Job], service: list[float]) -> np.ndarray:
    """Latencies of a one-job-at-a-time FCFS server with the given service
    times (completion_i = max(arrival_i, completion_{i-1}) + service_i)."""
    done = 0.0
    lat = []
    for j, s in zip(jobs, service):
        done = max(done, j.arrival) + s
        lat.append(done - j.arrival)
    return np.array(lat)


def summarize(records: list[Record]) -> dict:
    lat = np.array([r.latency for r in records])
    q = np.array([r.queueing for r in records])
    upd = sum(4 * r.job.L ** 2 * r.job.nsteps for r in records if r.job.algo == "met")
    cells = sum(r.job.L ** 2 * r.job.nsteps for r in records if r.job.algo == "sw")
    span = max(r.completed for r in records) - min(r.t_ref for r in records)
    return {"jobs": len(records), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "queue_p50_s": float(np.percentile(q, 50)), "queue_p99_s": float(np.percentile(q, 99)),
            "makespan_s": span, "met_updates_per_ns": upd / span / 1e9, "sw_cell_steps_per_ns": cells / span / 1e9}
