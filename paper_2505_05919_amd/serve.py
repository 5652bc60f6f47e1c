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
    # the quantum's launches (and batch rebuilds), waiting for the GPU, retiring
    # finished jobs (observables, digests)
    phase_s: dict = field(default_factory=lambda: {"admit": 0.0, "launch": 0.0, "wait": 0.0, "retire": 0.0})

    def _members(self, runs: list) -> list:
        if self.schedule == "srpt":
            return _srpt(runs, self.fill_cells)
        return runs

    def run(self, jobs: list[Job], realtime: bool = True) -> list[Record]:
        """Serve `jobs` (sorted by arrival).  realtime: arrivals are released
        by the wall clock from the start of the call; otherwise all jobs are
        available at once (arrival times are still used for latencies).

        The loop keeps one quantum in flight: it enqueues quantum k + 1 (whose
        members are known on the host: every job's step count advances at
        enqueue time) before it waits for quantum k, and retires the jobs that
        quantum k finished while k + 1 runs.  Host work that touches a chain
        outside a quantum -- creation, batch descriptor uploads, observables
        and digests of finished jobs -- goes to a third stream, so that it
        never waits for the quantum in flight."""
        import hashlib

        import torch
        stream_b = torch.cuda.current_stream()
        stream_s = torch.cuda.Stream()             # default priority
        stream_r = torch.cuda.Stream()             # chain set-up and retirement
        pending = list(jobs)
        queue: list[Job] = []
        running: list[Running] = []                # admitted, steps left to enqueue
        used = 0
        batch = None
        batch_members: tuple = ()
        swb = None
        swb_members: tuple = ()
        inflight = None                            # (events, jobs it finishes, batches to close after it)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0     # noqa: E731

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
            with torch.cuda.stream(stream_r):
                for r in finishing:
                    r.chain.stream = stream_r      # its quanta are complete; nothing waits for k + 1
                    o = r.chain.obs()
                    hash_it = self.keep_digest and (self.digest_seeds is None or r.job.seed in self.digest_seeds)
                    dg = hashlib.sha256(r.chain.sigma.cpu().numpy().tobytes()).hexdigest() if hash_it else ""
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
            admitted = False
            while queue and held < self.max_slots:
                fp = footprint(queue[0])
                if used + fp > self.memory_budget and held:
                    break
                job = queue.pop(0)
                p = cvf.cvf_params_from_si(job.T, job.P, L=job.L, seed=job.seed)
                mask = cvf.CVF_ALGO_METROPOLIS | (cvf.CVF_ALGO_SW if job.algo == "sw" else 0)
                with torch.cuda.stream(stream_r):
                    ch = cvf.Chain(p, mask, stream=stream_r)
                    ch.set_stop(job.nsteps)            # quanta may overshoot; the chain stops exactly
                ch.stream = stream_s if job.algo == "sw" else stream_b
                running.append(Running(job, ch, 0, now(), job.arrival if realtime else 0.0))
                admitted = True
                used += fp
                held += 1
                self.peak_resident_bytes = max(self.peak_resident_bytes, used)
                self.peak_resident_jobs = max(self.peak_resident_jobs, held)
            if admitted:
                stream_r.synchronize()                 # new chains are set up before their first quantum
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
            stale = []
            events = []
            # one quantum: every member advances by min(quantum, remaining) steps
            if met:
                steps = min(self.quantum, max(r.job.nsteps - r.done for r in met))
                members = tuple(id(r) for r in met)
                if members != batch_members:
                    if batch is not None:
                        stale.append(batch)            # closed once the quantum in flight is done
                    batch = cvf.Batch([r.chain for r in met], stream=stream_r)
                    batch.stream = stream_b
                    batch_members = members
                batch.metropolis(steps, graph_block=self.graph_block if steps % max(1, self.graph_block) == 0 else 0)
                events.append(torch.cuda.Event())
                events[-1].record(stream_b)
                for r in met:
                    r.done = min(r.done + steps, r.job.nsteps)
            if sws:
                n = min(self.quantum, max(r.job.nsteps - r.done for r in sws))
                members = tuple(id(r) for r in sws)
                if members != swb_members:
                    if swb is not None:
                        stale.append(swb)
                    swb = cvf.Batch([r.chain for r in sws], stream=stream_r)
                    swb.stream = stream_s
                    swb_members = members
                swb.sw(n)
                events.append(torch.cuda.Event())
                events[-1].record(stream_s)
                for r in sws:
                    r.done = min(r.done + n, r.job.nsteps)
            finishing = [r for r in running if r.done >= r.job.nsteps]
            running = [r for r in running if r.done < r.job.nsteps]
            if finishing:
                # a finished job leaves its batch: rebuild at the next quantum
                if any(r.job.algo == "met" for r in finishing):
                    batch_members = ()
                if any(r.job.algo == "sw" for r in finishing):
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
