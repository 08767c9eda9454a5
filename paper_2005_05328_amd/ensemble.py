"""Run control of a batched ensemble (many independent boxes in one particle state): DZS
coarsening box by box in place, re-packing of the survivors into a state fitted to the new
count, and the halt predicate of the paper's run control (Sec. 4.1.1) that decides when to
re-pack.  Marshalling only: the coarsening is the library's dzs_coarsen on each box's range,
the re-pack is device copies.

Layout: box b owns particles first[b] .. first[b+1] of the state (as kdk_step_batch expects).
"""
from __future__ import annotations

from . import _abi, State, halt_check

_ARR = ("x", "y", "z", "px", "py", "pz", "gx", "gy", "gz", "mult", "id", "type")


class _BoxRange:
    """A view of one box's particle range of a batched state (what dzs_coarsen reads and
    reorders in place); n follows the call's report."""

    def __init__(self, st: State, lo: int, hi: int):
        self.st, self.lo, self.n = st, lo, hi - lo
        self.capacity = hi - lo

    def view(self) -> _abi.Particles:
        p = _abi.Particles()
        for k in _ARR:
            t = getattr(self.st, k)
            setattr(p, k, t.data_ptr() + self.lo * t.element_size())
        p.n = self.n
        p.capacity = self.capacity
        return p


def coarsen_boxes(ctx, boxes, st: State, first, params):
    """DZS coarsening of every box of a batch, each in its own range (the survivors of box b
    end up in first[b] .. first[b] + counts[b], in (key, id) order).  params[b] is box b's
    CoarsenParams (None: the box is left as it is).  Returns (counts, reports)."""
    counts, reports = [], []
    for b, (box, prm) in enumerate(zip(boxes, params)):
        lo, hi = int(first[b]), int(first[b + 1])
        if prm is None or hi == lo:
            counts.append(hi - lo)
            reports.append(None)
            continue
        r = _BoxRange(st, lo, hi)
        reports.append(ctx.dzs_coarsen(box, r, prm))
        counts.append(r.n)
    return counts, reports


def repack(st: State, first, counts, capacity: int | None = None, device="cuda:0"):
    """The survivors of every box (first[b] .. first[b] + counts[b]) copied into a new state
    of capacity `capacity` (default: exactly their total), boxes in the same order.  Returns
    (new state, new first)."""
    new_first = [0]
    for c in counts:
        new_first.append(new_first[-1] + int(c))
    n = new_first[-1]
    out = State(capacity or max(n, 1), device)
    for k in _ARR:
        src, dst = getattr(st, k), getattr(out, k)
        for b, c in enumerate(counts):
            if c:
                dst[new_first[b]: new_first[b] + c].copy_(src[int(first[b]): int(first[b]) + c])
    out.n = n
    return out, new_first


def control(counts, n_last_pack: int, t: float = 1.0, t_prev: float = 0.0,
            ratio_prev: float = 1.0, min_ratio: float = 0.9, balance: float = 1.0,
            max_balance: float = 0.0, runtime_limit_s: float = 0.0,
            restart_window_s: float = 0.0):
    """The halt predicate on the ensemble's count against the count at the last packing:
    R = sum(counts) / n_last_pack.  Returns (R, the DZS_HALT_* reasons; re-pack when
    non-zero)."""
    ratio = sum(int(c) for c in counts) / float(n_last_pack)
    reasons = halt_check(balance=balance, ratio=ratio, ratio_prev=ratio_prev, t=t, t_prev=t_prev,
                         max_balance=max_balance, min_ratio=min_ratio,
                         runtime_limit_s=runtime_limit_s, restart_window_s=restart_window_s)
    return ratio, reasons
