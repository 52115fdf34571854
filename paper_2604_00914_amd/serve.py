"""Request loop over the native continuous-batching server (afsi_server_* in afsi.h).

The server (C++, in libafsi.so) owns admission, batching and the per-pool
worker threads; this module only feeds it a timed request stream, collects
completions and reports latency percentiles beside throughput.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import afsi


@dataclass
class Completed:
    rid: int
    tag: object
    eigenvalues: np.ndarray
    residuals: np.ndarray
    info: dict
    latency: float


@dataclass
class StreamReport:
    completed: list = field(default_factory=list)
    wall_s: float = 0.0
    stats: dict = field(default_factory=dict)

    def summary(self) -> dict:
        lat = np.array([c.latency for c in self.completed]) if self.completed else np.zeros(1)
        pairs = sum(len(c.eigenvalues) for c in self.completed)
        return {
            "requests": len(self.completed),
            "wall_s": round(self.wall_s, 3),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "mean_latency_s": round(float(lat.mean()), 4),
            "throughput_req_per_s": round(len(self.completed) / max(self.wall_s, 1e-9), 3),
            "eigenpairs_per_s": round(pairs / max(self.wall_s, 1e-9), 2),
            "slices_per_batched_launch": round(self.stats.get("batched_groups", 0) /
                                               max(self.stats.get("batched_launches", 1), 1), 3),
            # slice products that shared a grouped-kernel launch, per launch, and the share
            # of all slice products that went through the grouped kernel
            "slices_per_grouped_kernel": round(self.stats.get("kernel_slices", 0) /
                                               max(self.stats.get("kernel_launches", 1), 1), 3),
            "grouped_kernel_share": round(self.stats.get("kernel_slices", 0) /
                                          max(self.stats.get("batched_groups", 1), 1), 3),
        }


class Server:
    """Owns an afsi_server_t; matrices registered here stay resident until close()."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 200 << 30):
        self.handle = afsi.afsi_server_create(device, hbm_budget_bytes)
        self.device = device

    def set_pool_columns(self, matrix: afsi.Matrix, cols: int):
        afsi.afsi_server_set_pool_columns(self.handle, matrix.handle, cols)

    def submit(self, matrix: afsi.Matrix, a, b, p, opts, seed) -> int:
        return afsi.afsi_server_submit(self.handle, matrix.handle, a, b, p, opts, seed)

    def wait(self, rid, timeout_s=600.0):
        return afsi.afsi_server_wait(self.handle, rid, timeout_s)

    def wait_any(self, timeout_s):
        return afsi.afsi_server_wait_any(self.handle, timeout_s)

    def info(self, rid):
        return afsi.afsi_server_info(self.handle, rid)

    def fetch(self, rid, capacity, evecs=None):
        return afsi.afsi_server_fetch(self.handle, rid, capacity, evecs)

    def stats(self) -> dict:
        st = afsi.afsi_server_get_stats(self.handle)
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self):
        if self.handle:
            afsi.afsi_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def info_dict(info) -> dict:
    return {name: getattr(info, name) for name, _ in info._fields_}


def run_stream(server: Server, jobs, timeout_s: float = 3600.0) -> StreamReport:
    """Submit `jobs` at their arrival times and collect every completion.

    jobs: iterable of (arrival_s, matrix, a, b, p, opts, seed, tag), sorted by arrival.
    Latency is completion minus submission on the server's clock.
    """
    jobs = list(jobs)
    report = StreamReport()
    tags = {}
    lock = threading.Lock()
    submitted = threading.Event()
    errors = []

    def collector():
        remaining = None
        while True:
            with lock:
                if submitted.is_set():
                    remaining = len(jobs) - len(report.completed)
            if remaining == 0:
                return
            rid = server.wait_any(0.5)
            if rid < 0:
                continue
            try:
                info = server.info(rid)
                lam, res = server.fetch(rid, capacity=max(int(info.count), 1))
                with lock:
                    report.completed.append(Completed(rid, tags.get(rid), lam, res, info_dict(info),
                                                      info.t_done - info.t_submit))
            except Exception as e:  # surfaced after the stream
                errors.append(e)
                with lock:
                    report.completed.append(Completed(rid, tags.get(rid), np.zeros(0), np.zeros(0), {}, float("nan")))

    th = threading.Thread(target=collector, daemon=True)
    t0 = time.perf_counter()
    th.start()
    for (arrival, matrix, a, b, p, opts, seed, tag) in jobs:
        delay = arrival - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        with lock:  # the collector reads a request's tag under this lock
            rid = server.submit(matrix, a, b, p, opts, seed)
            tags[rid] = tag
    submitted.set()
    th.join(timeout_s)
    report.wall_s = time.perf_counter() - t0
    report.stats = server.stats()
    if errors:
        raise errors[0]
    return report
