"""The benchmark's accuracy report (no GPU): errors planted in outputs held as CPU
tensors come back as planted, on the oracle's own sample of the workload."""
import numpy as np
import pytest

import oracle
from paper_2601_18548_amd import workloads as wl

torch = pytest.importorskip("torch")


def test_accuracy_report_recovers_planted_errors():
    import bench

    wk = wl.workload("small")
    dr, Jr = oracle.eval_grad(wk.weights.to_blob(), wk.knots, wk.points)
    d = torch.from_numpy((dr + 1e-4).astype(np.float32))
    J = torch.from_numpy((Jr * (1 + 2e-3)).astype(np.float32))
    base, acc = bench.cpu_baseline(wk, 0.2, torch, d, J)
    assert base["kind"] == "oracle" and base["value"] > 0 and acc["pairs"] > 0
    assert abs(acc["max_abs_dd"] - 1e-4) < 2e-6 and abs(acc["mean_abs_dd"] - 1e-4) < 2e-6
    assert abs(acc["max_rel_J"] - 2e-3) < 1e-5 and abs(acc["mean_rel_J"] - 2e-3) < 1e-5
