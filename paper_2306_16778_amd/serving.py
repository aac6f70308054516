"""Replay of a request trace through the queued serving entry points.

Requests exp(t_i A_i) v_i arrive as a Poisson process (workloads.config5_requests).
The replay keeps a look-ahead window of prepared requests: each new matrix is
assembled on the GPU on a preparation stream and registered with the queue (a
stream-ordered copy), its vector copied and its output allocated, while the
submitting loop waits for the next arrival time.  Registered matrices are
released least-recently-used first once they exceed a resident-bytes cap; a
later request for a released matrix assembles and registers it again.  The
queue (the C++ scheduler inside libexpm_pfd) does admission by HBM budget,
grouping and launches; this module only paces submissions and collects the
statistics.
"""

from __future__ import annotations

import collections
import sys
import time

import numpy as np

from . import expm_pfd as ep
from . import workloads


class _Prepared:
    __slots__ = ("req", "mat", "V", "X", "ev")

    def __init__(self, req, mat, V, X, ev):
        self.req, self.mat, self.V, self.X, self.ev = req, mat, V, X, ev


def replay(count: int, qps: float, precision: str = "mixed", degree: int = 16, n_lo: int = 64, n_hi: int = 4096,
           budget_bytes: int = 64 << 30, max_group: int = 64, streams: int = 3, keep=None,
           resident_bytes: int | None = None, lookahead: int = 48, at_once: bool = False, progress_s: float = 0.0,
           reqs=None, specs=None):
    """Submit ``count`` requests at their arrival times (``at_once``: all prepared first,
    then submitted back to back at time 0, a closed-loop saturation run) and wait for
    all of them.

    keep: optional predicate on a request; for those, (request, v, t, X host copy) are returned
    so results can be checked.  resident_bytes: cap on registered matrix bytes (default: half
    the budget).  progress_s > 0 prints a progress line to stderr that often.
    Returns (stats dict, kept list, wall seconds, late submissions)."""
    import torch

    if reqs is None:
        reqs, specs = workloads.config5_requests(count, qps, n_lo, n_hi)
    reqs = reqs[:count]
    cap = resident_bytes if resident_bytes is not None else (budget_bytes * 3) // 5 if at_once else budget_bytes // 2
    q = ep.expm_pfd_queue_create(budget_bytes, degree, precision, max_group=max_group, streams=streams)
    prep = torch.cuda.Stream()  # matrix assembly, registration copies, vector copies
    sub = torch.cuda.Stream()   # carries each request's readiness to the queue
    resident = collections.OrderedDict()  # matrix index -> (queue id, bytes, pending submissions)
    resident_sum = 0
    window = collections.deque()
    kept = []
    late = 0
    nxt = 0

    def evict(limit=None):
        nonlocal resident_sum
        limit = cap if limit is None else limit
        for key in list(resident):
            if resident_sum <= limit:
                break
            mid, nbytes, pins = resident[key]
            if pins:
                continue  # a prepared request still names it
            ep.expm_pfd_unregister_matrix(q, mid)
            resident_sum -= nbytes
            del resident[key]

    def prepare(r):
        nonlocal resident_sum
        with torch.cuda.stream(prep):
            if r.matrix_id in resident:
                mid, nbytes, pins = resident.pop(r.matrix_id)
            else:
                A = workloads.config5_matrix_device(specs[r.matrix_id])
                for attempt in range(100000):
                    try:
                        mid = ep.expm_pfd_register_matrix(q, A, stream=prep)
                        break
                    except ep.ExpmPfdError as e:
                        # the budget (or the device) is full of work in flight: release
                        # what can be released and let some of it complete
                        if e.code not in (-9, -5) or attempt == 99999:
                            raise
                        evict(0)
                        time.sleep(1e-3)
                nbytes = r.n * r.n * 16
                resident_sum += nbytes
                pins = 0
            resident[r.matrix_id] = (mid, nbytes, pins + 1)  # most recently used last
            V = torch.from_numpy(np.asfortranarray(r.v)).pin_memory().to("cuda", non_blocking=True)
            X = torch.empty((r.v.shape[1], r.n), dtype=torch.complex128, device="cuda").t()
            ev = torch.cuda.Event()
            ev.record(prep)
        evict()
        return _Prepared(r, mid, V, X, ev)

    if at_once:
        # closed loop: every request prepared first, then all submitted back to back
        while nxt < len(reqs):
            window.append(prepare(reqs[nxt]))
            nxt += 1
        prep.synchronize()
    t0 = time.perf_counter()
    last_print = 0.0
    for k, r in enumerate(reqs):
        # prepare ahead while the next arrival is not yet due
        while nxt < len(reqs) and (nxt <= k or (len(window) < lookahead and
                                               r.arrival_s - (time.perf_counter() - t0) > 2e-3)):
            window.append(prepare(reqs[nxt]))
            nxt += 1
        if not at_once:
            wait = r.arrival_s - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            elif wait < -1e-3:
                late += 1
        p = window.popleft()
        sub.wait_event(p.ev)
        tk, _ = ep.expm_pfd_submit(q, p.mat, p.req.t, p.V, p.X, stream=sub)
        key = p.req.matrix_id
        mid, nbytes, pins = resident[key]
        resident[key] = (mid, nbytes, pins - 1)
        if keep is not None and keep(p.req):
            kept.append((p.req, p.X))
        if progress_s > 0:
            now = time.perf_counter() - t0
            if now - last_print >= progress_s:
                last_print = now
                st = ep.expm_pfd_queue_stats_get(q)
                print(f"[serving {precision}] {k + 1}/{len(reqs)} submitted, {st['completed']} completed, "
                      f"{now:.1f} s", file=sys.stderr, flush=True)
    for mid, _, _ in resident.values():  # freed as their last requests complete
        ep.expm_pfd_unregister_matrix(q, mid)
    resident.clear()
    ep.expm_pfd_queue_drain(q)
    wall = time.perf_counter() - t0
    stats = ep.expm_pfd_queue_stats_get(q)
    out = [(r, r.v, r.t, X.cpu().numpy()) for r, X in kept]
    ep.expm_pfd_queue_destroy(q)
    # hand torch's cached blocks (assembled matrices, vectors) back to the device
    # so that a later queue's stream-ordered pool finds the memory
    del window, resident
    torch.cuda.empty_cache()
    return stats, out, wall, late
