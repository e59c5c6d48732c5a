"""Host checks of bench.py's contract pieces that need no GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_model_op_count_matches_the_per_pair_model():
    # n = 8, d = 3: 192 lines x 28 unique pairs x 65 + 1536 diagonal fluxes x 25
    assert bench.model_ops_per_element(8) == 192 * 28 * 65 + 1536 * 25 == 387840


def test_profile_counters_are_used_only_for_the_profiled_sources(monkeypatch, tmp_path):
    ctr = bench.profiled_counters()
    if ctr is not None:
        assert ctr["digest"] == bench.kernel_source_digest()
        assert ctr["fetch_kib"] > 0 and ctr["write_kib"] > 0
    # a different kernel source gives a different digest and no counters
    other = tmp_path / "k.hip"
    other.write_text("// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(other)])    # absolute: joined paths ignore ROOT
    assert os.path.exists(os.path.join(bench.ROOT, bench.TRAFFIC_PROFILE))
    assert bench.profiled_counters() is None


def test_smooth_state_stays_physical_on_other_nodes(orc):
    """The over-integrated leg's input: interpolated from the 8 GL nodes to
    10 (modes P, then V on the 10 nodes), density and pressure stay positive;
    the generator is deterministic in its seed."""
    from paper_2306_11665_amd import workloads as W
    n, m, E = 8, 10, 64
    u = W.smooth_euler_state(E, n, seed=11)
    assert np.array_equal(u, W.smooth_euler_state(E, n, seed=11))
    _, Pn = orc.basis_rect(n, n, "gl")
    Vm, _ = orc.basis_rect(n, m, "gl")
    uq = orc.tensor_apply(orc.tensor_apply(u, n, 3, Pn), n, 3, Vm)
    rho = uq[0]
    p = 0.4 * (uq[4] - 0.5 * (uq[1] ** 2 + uq[2] ** 2 + uq[3] ** 2) / rho)
    assert rho.min() > 0.3 and p.min() > 0.3
