"""Replay of a request trace through the queued serving entry points.

Requests exp(t_i A_i) v_i arrive as a Poisson process (workloads.config5_requests);
matrices are assembled on the GPU when first seen, registered with the queue and
reused by later requests with a new t.  The queue (C++ scheduler inside
libexpm_pfd) does admission by HBM budget, grouping and launches; this module
only paces the submissions and collects the statistics.
"""

from __future__ import annotations

import time

import numpy as np

from . import expm_pfd as ep
from . import workloads


def replay(count: int, qps: float, precision: str = "mixed", degree: int = 16, n_lo: int = 64, n_hi: int = 4096,
           budget_bytes: int = 64 << 30, max_group: int = 64, streams: int = 3, keep=None):
    """Submit ``count`` requests at their arrival times and wait for all of them.

    keep: optional predicate on a request; for those, (A host copy, v, t, X device) are returned
    so results can be checked.  Returns (stats dict, kept list, wall seconds)."""
    import torch

    reqs, specs = workloads.config5_requests(count, qps, n_lo, n_hi)
    q = ep.expm_pfd_queue_create(budget_bytes, degree, precision, max_group=max_group, streams=streams)
    mat_ids, mats = {}, {}
    kept = []
    t0 = time.perf_counter()
    for r in reqs:
        if r.matrix_id not in mat_ids:
            A = workloads.config5_matrix_device(specs[r.matrix_id])
            mat_ids[r.matrix_id] = ep.expm_pfd_register_matrix(q, A)
            mats[r.matrix_id] = A
        V = torch.from_numpy(np.asfortranarray(r.v)).to("cuda")
        now = time.perf_counter() - t0
        if r.arrival_s > now:
            time.sleep(r.arrival_s - now)
        _, X = ep.expm_pfd_submit(q, mat_ids[r.matrix_id], r.t, V)
        if keep is not None and keep(r):
            kept.append((r, mats[r.matrix_id], r.v, r.t, X))
        # the queue holds its own copy of every registered matrix; the caller's copies are only
        # kept when results are to be checked (a later request may reuse any earlier matrix)
        if keep is None and len(mats) > 8:
            for k in list(mats)[:-8]:
                del mats[k]
    ep.expm_pfd_queue_drain(q)
    wall = time.perf_counter() - t0
    stats = ep.expm_pfd_queue_stats_get(q)
    out = [(r, A.cpu().numpy(), v, t, X.cpu().numpy()) for r, A, v, t, X in kept]
    ep.expm_pfd_queue_destroy(q)
    return stats, out, wall
