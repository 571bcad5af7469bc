"""Helpers for the GPU parity tests: device transfer and walk comparison
against the oracle under the boundary tolerance."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

BOUNDARY_TOL = 1e-6
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# every labelled comparison appends its counts here (one JSON object a line),
# so that a GPU run leaves the boundary-mismatch rate of each case behind
MISMATCH_LOG = os.path.join(ROOT, "gpurun_out", "parity_mismatch.jsonl")


def record_mismatch(label: str, kind: str, walks: int, identical: int, boundary: int):
    os.makedirs(os.path.dirname(MISMATCH_LOG), exist_ok=True)
    with open(MISMATCH_LOG, "a") as fh:
        fh.write(json.dumps({"case": label, "kind": kind, "walks": int(walks),
                             "identical": int(identical), "boundary": int(boundary),
                             "rate": boundary / max(int(walks), 1)}) + "\n")


def gpu_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_16182_amd as tw
    tw.lib()  # raises when the library is not built: the HIP path must be there
    return torch, tw


def to_dev(torch, *arrays):
    dev = torch.device("cuda", 0)
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrays]


def compare_walks(gpu, orc, exact: bool, label: str = None, kind: str = None):
    """gpu: (nodes, ts, len) numpy; orc: oracle result with margins.

    Returns (identical, boundary) counts; asserts that every non-identical
    walk first differs at a position whose pick sat within BOUNDARY_TOL of an
    exponential CDF boundary (never for exact pickers). With a label, the
    counts are appended to the mismatch log."""
    gn, gt, gl = gpu
    on, ot, ol = orc["nodes"], orc["ts"], orc["len"]
    assert gn.shape == on.shape
    eq = (gn == on) & (gt == ot)
    same = eq.all(1) & (gl == ol)
    bad = np.flatnonzero(~same)
    boundary = 0
    for i in bad:
        k = int(np.argmin(eq[i])) if not eq[i].all() else int(min(gl[i], ol[i]))
        m = orc["margin"][i, k] if orc.get("margin") is not None and k < on.shape[1] else 0.0
        assert not exact and m < BOUNDARY_TOL, (
            f"walk {i} differs at position {k} (margin {m}): gpu {gn[i][:gl[i]]} "
            f"oracle {on[i][:ol[i]]}")
        boundary += 1
    if label is not None:
        record_mismatch(label, kind or "", len(gl), int(same.sum()), boundary)
    return int(same.sum()), boundary
