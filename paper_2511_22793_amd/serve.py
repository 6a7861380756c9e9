"""Batched serving of uneven queries: many receivers over several scenes of
different Gaussian count, grid and channel count, rendered by one persistent
blend launch (include/gsparc.h, gs_batch_*) that can be captured in a HIP
graph, with tile shapes, channel groups and the persistent grid chosen by an
autotuner.

  Job       one scene, its attributes and a group of receivers
  Batch     device buffers (spectra, workspaces, plan, timestamps) for a
            list of jobs; run() enqueues, capture() records a graph,
            replay() launches it, latencies_ms() reads the device timestamps
  Autotuner per-job tile shape and channel group by timing each candidate on
            a few of the job's queries, the workgroup size class minimising
            the summed job times, then the persistent workgroup count on the
            whole batch; results cached per job signature
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np
import torch

from ._lib import GsBatchInfo, GsBatchJob, GsQueries, check, lib
from .render import Grid, Params, Workspace, _attrs_c, _check_f32, _ptr, _scene_c, fit_pair_capacity


@dataclass
class Job:
    """A scene (dict of float32 device tensors), attributes shared by its
    receivers ([n,F] real or [n,F,2] complex) or per receiver ([B,n,F(,2)]),
    and receivers rx [B,3]."""
    scene: dict
    attr: torch.Tensor
    rx: torch.Tensor
    is_complex: bool = False
    grid: Grid = field(default_factory=Grid)
    params: Params = field(default_factory=lambda: Params(forward_only=True))
    tx: Optional[torch.Tensor] = None

    @property
    def n(self):
        return int(self.scene["opacity_logit"].shape[0])

    @property
    def B(self):
        return int(self.rx.shape[0])

    @property
    def F(self):
        return int(self.attr.shape[-2] if self.is_complex else self.attr.shape[-1])

    def signature(self) -> str:
        return "n%d_%dx%d_F%d%s" % (self.n, self.grid.H, self.grid.W, self.F, "c" if self.is_complex else "r")

    def head(self, k: int) -> "Job":
        """The same job on its first k receivers."""
        k = min(k, self.B)
        per_set = self.attr.dim() == (4 if self.is_complex else 3)
        return replace(self, rx=self.rx[:k].contiguous(), attr=self.attr[:k].contiguous() if per_set else self.attr,
                       tx=None if self.tx is None else self.tx[:k].contiguous())


class Batch:
    """Device state of one batch; the jobs' order is the service order."""

    def __init__(self, jobs: list, workgroups: Optional[int] = None, device=None, fit_capacity: bool = True):
        """fit_capacity: size each job's pair buffer from one prepare of its
        queries (fit_pair_capacity; jobs whose params already set
        pair_capacity keep it)."""
        if not jobs:
            raise ValueError("a batch needs at least one job")
        if fit_capacity:
            jobs = [replace(j, params=fit_pair_capacity(j.scene, j.rx, j.tx, j.grid, j.params))
                    if j.params.pair_capacity == 0 else j for j in jobs]
        self.jobs = list(jobs)
        dev = device or jobs[0].rx.device
        self.device = dev
        self.spectra, self.workspaces = [], []
        self._cjobs = (GsBatchJob * len(jobs))()
        for i, j in enumerate(self.jobs):
            _check_f32("rx", j.rx, (j.B, 3))
            if j.tx is not None:
                _check_f32("tx", j.tx, (j.B, 3))
            shape = (j.B, j.F, j.grid.H, j.grid.W) + ((2,) if j.is_complex else ())
            out = torch.empty(shape, dtype=torch.float32, device=dev)
            ws = Workspace(j.n, j.B, j.grid, j.params, device=dev)
            self.spectra.append(out)
            self.workspaces.append(ws)
            c = self._cjobs[i]
            c.scene = _scene_c(j.scene)
            c.attrs = _attrs_c(j.attr, j.n, j.B, j.is_complex)
            c.queries = GsQueries(j.B, _ptr(j.rx), _ptr(j.tx))
            c.grid = j.grid.c()
            c.params = j.params.c()
            c.spectrum = _ptr(out)
            c.workspace = ctypes.c_void_p(ws.ptr)
            c.workspace_bytes = ws.nbytes
        L = lib()
        self.plan_bytes = L.gs_batch_plan_bytes(len(jobs))
        self._plan = torch.empty(self.plan_bytes + 256, dtype=torch.uint8, device=dev)
        self.plan_ptr = self._plan.data_ptr() + (-self._plan.data_ptr()) % 256
        self.info = GsBatchInfo()
        stream = torch.cuda.current_stream(dev).cuda_stream
        check(L.gs_batch_plan(self._cjobs, len(jobs), ctypes.c_void_p(self.plan_ptr), self.plan_bytes,
                              ctypes.byref(self.info), ctypes.c_void_p(stream)), "gs_batch_plan")
        self.n_queries = self.info.n_queries
        self.workgroups = int(workgroups) if workgroups else int(self.info.workgroups)
        self.timestamps = torch.zeros(self.n_queries + 3, dtype=torch.int64, device=dev)
        khz = ctypes.c_int32()
        check(L.gs_wall_clock_khz(ctypes.byref(khz)), "gs_wall_clock_khz")
        self.clock_khz = khz.value
        self.graph = None

    def run(self, timestamps: bool = True):
        """Enqueues the whole batch on the current stream."""
        stream = torch.cuda.current_stream(self.device).cuda_stream
        ts = ctypes.c_void_p(self.timestamps.data_ptr()) if timestamps else None
        check(lib().gs_batch_run(self._cjobs, len(self.jobs), ctypes.c_void_p(self.plan_ptr), self.plan_bytes,
                                 self.workgroups, ts, ctypes.c_void_p(stream)), "gs_batch_run")

    def capture(self) -> torch.cuda.CUDAGraph:
        """Records run() into a graph (one eager run first, as warm-up)."""
        self.run()
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def latencies_ms(self) -> dict:
        """Per-query latency (completion - batch start, ms, job order) and
        the batch makespan, from the device timestamps of the last run."""
        ts = self.timestamps.cpu().numpy().astype(np.float64)
        per_tick = 1.0 / self.clock_khz  # ms
        nq = self.n_queries
        lat = (ts[1:nq + 1] - ts[0]) * per_tick
        return {"per_query": lat, "makespan": (ts[nq + 1] - ts[0]) * per_tick,
                "prepare": (ts[nq + 2] - ts[0]) * per_tick,
                "p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}

    def flags(self):
        return [ws.flags() for ws in self.workspaces]


TILE_SHAPES = {256: ((16, 16), (8, 32), (32, 8)), 128: ((8, 16), (16, 8)), 64: ((8, 8),)}
CHAN_GROUPS = (8, 16, 32)


def _time(fn, reps: int) -> float:
    """Median ms of fn() over reps runs (HIP events on the current stream)."""
    fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


class Autotuner:
    """Chooses, per job, the tile shape (rows x columns) and the channel
    group, then one workgroup size class for the batch and the number of
    persistent workgroups.

    Per job signature (Gaussian count, grid, channels): every candidate
    shape of each class and every channel group dividing F*c is timed on the
    job's first `probe` receivers as a one-job batch; the best per class is
    kept (cached in `cache`, a JSON file when `path` is given).  The class
    whose summed best times over the batch is smallest wins, then the
    workgroup count (fractions of the full-occupancy count) is timed on the
    whole batch.  Jobs are ordered shortest estimated time first."""

    def __init__(self, path: Optional[str] = None, probe: int = 4, reps: int = 3,
                 wg_fractions=(1.0, 0.75, 0.5)):
        self.path, self.probe, self.reps, self.wg_fractions = path, probe, reps, wg_fractions
        self.cache = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)
        self.log = []

    def _save(self):
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)

    def tune_job(self, job: Job) -> dict:
        key = job.signature()
        if key in self.cache:
            return self.cache[key]
        probe = job.head(self.probe)
        fc = job.F * (2 if job.is_complex else 1)
        groups = [c for c in CHAN_GROUPS if fc % c == 0] or [fc & -fc if fc & -fc <= 32 else 32]
        res = {}
        for block, shapes in TILE_SHAPES.items():
            best = None
            for th, tw in shapes:
                for cg in groups:
                    grid = replace(job.grid, tile_h=th, tile_w=tw)
                    params = replace(job.params, chan_group=cg)
                    b = Batch([replace(probe, grid=grid, params=params)])
                    ms = _time(lambda: b.run(timestamps=False), self.reps) / probe.B
                    self.log.append((key, th, tw, cg, ms))
                    if best is None or ms < best["ms_per_query"]:
                        best = {"tile_h": th, "tile_w": tw, "chan_group": cg, "ms_per_query": ms}
                    del b
            res[str(block)] = best
        self.cache[key] = res
        self._save()
        return res

    def tune(self, jobs: list, tune_workgroups: bool = True) -> Batch:
        """Returns a Batch of the tuned, reordered jobs."""
        per = [self.tune_job(j) for j in jobs]
        totals = {blk: sum(p[str(blk)]["ms_per_query"] * j.B for p, j in zip(per, jobs)) for blk in TILE_SHAPES}
        blk = min(totals, key=totals.get)
        tuned = []
        for p, j in zip(per, jobs):
            c = p[str(blk)]
            tuned.append((c["ms_per_query"] * j.B,
                          replace(j, grid=replace(j.grid, tile_h=c["tile_h"], tile_w=c["tile_w"]),
                                  params=replace(j.params, chan_group=c["chan_group"]))))
        tuned.sort(key=lambda t: t[0])  # shortest job first
        batch = Batch([t[1] for t in tuned])
        self.choice = {"block": blk, "jobs": [(t[1].signature(), t[1].grid.tile_h, t[1].grid.tile_w,
                                               t[1].params.chan_group) for t in tuned]}
        if tune_workgroups:
            full = batch.info.workgroups
            best = None
            for frac in self.wg_fractions:
                batch.workgroups = max(1, int(full * frac))
                ms = _time(lambda: batch.run(timestamps=False), self.reps)
                if best is None or ms < best[1]:
                    best = (batch.workgroups, ms)
            batch.workgroups = best[0]
            self.choice["workgroups"] = best[0]
        return batch


def make_jobs(specs: list, device="cuda") -> list:
    """Jobs from host arrays: specs of (scene dict, attr, rx, is_complex, H, W)."""
    jobs = []
    for sc, attr, rx, cplx, H, W in specs:
        scene = {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(device) for k, v in sc.items()}
        jobs.append(Job(scene, torch.from_numpy(np.ascontiguousarray(attr, np.float32)).to(device),
                        torch.from_numpy(np.ascontiguousarray(rx, np.float32)).to(device), bool(cplx), Grid(H, W)))
    return jobs
