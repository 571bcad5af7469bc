"""Helpers for the GPU parity tests: device transfer and walk comparison
against the oracle under the boundary tolerance."""
from __future__ import annotations

import numpy as np
import pytest

BOUNDARY_TOL = 1e-6


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


def compare_walks(gpu, orc, exact: bool):
    """gpu: (nodes, ts, len) numpy; orc: oracle result with margins.

    Returns (identical, boundary) counts; asserts that every non-identical
    walk first differs at a position whose pick sat within BOUNDARY_TOL of an
    exponential CDF boundary (never for exact pickers)."""
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
    return int(same.sum()), boundary
