"""Checkpoint and resume of a time integration with the library.

A cRKFR step is a one-step method: the state u^n, the time reached and the
step count are all a run needs to continue (dt, the GLM cleaning speed and
the blending coefficients of the next step are functions of u^n, which
crk_prepare recomputes on resume, bit for bit as the pipelined step left
them).  The file holds

    8 bytes  b"CRKCKPT1"
    8 bytes  little-endian length L of the header
    L bytes  JSON header: format version, the solver's constructor arguments,
             state shape and dtype, t, step, the dt and c_h at the time of
             saving (for information), the SHA-256 of the state bytes, and
             any user entries
    the state u[v][e][node] as raw little-endian FP64 or FP32, C order

and nothing else, so that other tools can read it with a few lines.  A
trained network bound to the solver is saved beside it with MLP.save.
"""
from __future__ import annotations

import hashlib
import json
import os
import struct

import numpy as np

MAGIC = b"CRKCKPT1"
VERSION = 1


def write_file(path: str, header: dict, state: np.ndarray) -> None:
    """Write the checkpoint file format (host array; atomic rename)."""
    state = np.ascontiguousarray(state)
    if state.dtype not in (np.float64, np.float32):
        raise ValueError("state must be float64 or float32")
    raw = state.astype(state.dtype.newbyteorder("<"), copy=False).tobytes(order="C")
    head = dict(header)
    head.update(version=VERSION, shape=list(state.shape), dtype=str(state.dtype),
                sha256=hashlib.sha256(raw).hexdigest())
    hb = json.dumps(head, sort_keys=True).encode()
    tmp = path + ".tmp"
    with open(tmp, "wb") as fh:
        fh.write(MAGIC)
        fh.write(struct.pack("<Q", len(hb)))
        fh.write(hb)
        fh.write(raw)
    os.replace(tmp, path)


def read_file(path: str):
    """(header, state) from a checkpoint file; the state's checksum and size
    are verified."""
    with open(path, "rb") as fh:
        if fh.read(8) != MAGIC:
            raise ValueError(f"{path}: not a checkpoint of this library")
        (n,) = struct.unpack("<Q", fh.read(8))
        head = json.loads(fh.read(n).decode())
        if head.get("version") != VERSION:
            raise ValueError(f"{path}: unsupported checkpoint version {head.get('version')}")
        raw = fh.read()
    dt = np.dtype(head["dtype"]).newbyteorder("<")
    count = int(np.prod(head["shape"]))
    if len(raw) != count * dt.itemsize:
        raise ValueError(f"{path}: state holds {len(raw)} bytes, expected {count * dt.itemsize}")
    if hashlib.sha256(raw).hexdigest() != head["sha256"]:
        raise ValueError(f"{path}: state checksum mismatch")
    state = np.frombuffer(raw, dtype=dt).reshape(head["shape"]).astype(head["dtype"])
    return head, state


def save(path: str, solver, u, t: float = 0.0, step: int = 0, dt=None, extra: dict | None = None) -> None:
    """Checkpoint state u (a device tensor of the solver's layout) at time t
    after `step` steps.  dt: the solver's dt buffer, recorded for information."""
    import torch
    solver._check_state(u)
    torch.cuda.synchronize(u.device)
    head = dict(config=solver.config, t=float(t), step=int(step))
    if dt is not None:
        d = dt.detach().cpu().numpy().astype(float)
        head.update(dt=float(d[0]), ch=float(d[1]))
    if extra:
        head["extra"] = extra
    write_file(path, head, u.detach().cpu().numpy())


def load(path: str, device: str = "cuda"):
    """Rebuild the solver and the state of a checkpoint.  Returns (solver,
    u, header); resume with solver.prepare(u, dt) and pipelined advances."""
    import torch
    from . import crk
    head, state = read_file(path)
    s = crk.Solver(device=device, **head["config"])
    if tuple(head["shape"]) != tuple(s.shape):
        raise ValueError(f"{path}: state shape {head['shape']} does not match the solver's {s.shape}")
    u = torch.from_numpy(np.ascontiguousarray(state)).to(device=device, dtype=s.dtype)
    return s, u, head
