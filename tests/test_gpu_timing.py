"""Phase timing of a solve (RS_SOLVE_TIMING): the events around every sketch and
factor change nothing the solver computes, and the three phase times are positive,
add up to no more than the host's own clock around the call, and stay 0 with the
flag off."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import make_problem, spectrum  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_05874_amd import rs as _rs
    _rs.load()
    yield _rs
    _rs.set_phase_timing(False)


def dev_padded(A, rs):
    dt = torch.float64 if A.dtype == np.float64 else torch.float32
    T = rs.padded(A.shape[0], A.shape[1], dtype=dt)
    T.copy_(torch.from_numpy(A))
    return T


def _problem(dtype, n=20000, d=300, seed=3):
    p = make_problem(n, d, spectrum("geom", d, 0.98), 1e-3, 0.1, seed, dtype=dtype)
    return p


def _phases(info):
    return info["ms_sketch"], info["ms_factor"], info["ms_iterate"]


@pytest.mark.parametrize("dtype,m_init", [(np.float64, 1), (np.float32, 1), (np.float32, 64)])
def test_timing_changes_nothing_and_adds_up(rs, dtype, m_init):
    p = _problem(dtype)
    A, b = dev_padded(p.A, rs), torch.from_numpy(p.b).cuda()
    rs.set_phase_timing(False)
    x0, i0 = rs.rs_adaptive_solve(A, b, p.nu2, seed=7, m_init=m_init)
    assert _phases(i0) == (0.0, 0.0, 0.0)
    rs.set_phase_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x1, i1 = rs.rs_adaptive_solve(A, b, p.nu2, seed=7, m_init=m_init)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    rs.set_phase_timing(False)
    assert torch.equal(x0, x1)
    assert i0["events"] == i1["events"] and i0["steps"] == i1["steps"]
    sk, fa, it = _phases(i1)
    assert sk > 0.0 and fa > 0.0 and it >= 0.0
    # the phases are parts of one GPU time line that the host clock encloses
    assert sk + fa + it <= wall_ms * 1.01 + 0.05


def test_timing_on_batches(rs):
    probs = [_problem(np.float32, n=6000 + 500 * i, d=120, seed=20 + i) for i in range(5)]
    dev_probs = [(dev_padded(p.A, rs), torch.from_numpy(p.b).cuda(), p.nu2) for p in probs]
    plain = rs.rs_solve_batch(dev_probs, seed=2, workers=3)
    rs.set_phase_timing(True)
    timed = rs.rs_solve_batch(dev_probs, seed=2, workers=3)
    rs.set_phase_timing(False)
    for (x0, i0), (x1, i1) in zip(plain, timed):
        assert torch.equal(x0, x1) and i0["events"] == i1["events"]
        assert _phases(i0) == (0.0, 0.0, 0.0)
        sk, fa, it = _phases(i1)
        assert sk > 0.0 and fa > 0.0 and it >= 0.0

