"""Checkpoint and restart of a run's particle state (host files, no part of the step).

A checkpoint holds every array of the state (positions, momenta, the force of the last step,
multiplicities, ids, types) in its current order, the count, and the caller's metadata (the
step index and scale factor reached, the run's parameters).  Restarting from it continues the
run bit for bit: a step reads nothing else that earlier steps left behind (the context keeps
only scratch and tables rebuilt from the step's arguments).
"""
from __future__ import annotations

import json

import numpy as np

ARRAYS = ("x", "y", "z", "px", "py", "pz", "gx", "gy", "gz", "mult", "id", "type")


def save(path: str, st, meta: dict | None = None) -> None:
    """Write the state (device) and `meta` (JSON-serialisable) to `path` (.npz)."""
    h = st.to_host()
    np.savez(path, n=np.int64(st.n), meta=np.frombuffer(json.dumps(meta or {}).encode(), np.uint8),
             **{k: h[k] for k in ARRAYS})


def load(path: str, capacity: int | None = None, device="cuda:0"):
    """(State on the device, meta) from a checkpoint written by save()."""
    from . import State
    with np.load(path, allow_pickle=False) as f:
        n = int(f["n"])
        st = State(capacity or max(n, 1), device)
        import torch
        for k in ("x", "y", "z", "px", "py", "pz", "gx", "gy", "gz"):
            getattr(st, k)[:n] = torch.from_numpy(f[k])
        st.mult[:n] = torch.from_numpy(f["mult"].view(np.int32))
        st.id[:n] = torch.from_numpy(f["id"].view(np.int32))
        st.type[:n] = torch.from_numpy(f["type"])
        st.n = n
        meta = json.loads(bytes(f["meta"]).decode())
    return st, meta
