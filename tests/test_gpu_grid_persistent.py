"""The nu grid's persistent form (RS_SOLVE_PERSISTENT): each window of steps of all
nu runs as one cooperative launch with grid barriers between its phases.  It
computes exactly what the separate launches compute, so every solution and every
record must equal the default form's bit for bit (FP64 and FP32, both variants,
both resample modes, uneven convergence across nu, check windows of 1 and 4),
and the full 2^18 x 2048 grid still reaches the oracle's solution."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ridge  # noqa: E402
from synth import config_c1, config_c4a_nu2, make_c4a_problem, make_problem, spectrum  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_05874_amd import rs as _rs
    _rs.load()
    return _rs


def dev_padded(A, rs):
    dt = torch.float64 if A.dtype == np.float64 else torch.float32
    T = rs.padded(A.shape[0], A.shape[1], dtype=dt)
    T.copy_(torch.from_numpy(A))
    return T


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


KEYS = ("status", "m_final", "doublings", "steps", "grad_passes", "accepted_polyak",
        "accepted_gd", "r_final", "events")


def same(rs, A, b, nus, **kw):
    print(f"[grid persistent] n={A.shape[0]} d={A.shape[1]} nu={len(nus)} {kw}", flush=True)
    X0, I0 = rs.rs_solve_nu_grid(A, b, nus, **kw)
    X1, I1 = rs.rs_solve_nu_grid(A, b, nus, persistent=True, **kw)
    assert torch.equal(X0, X1)
    for i0, i1 in zip(I0, I1):
        assert {k: i0[k] for k in KEYS} == {k: i1[k] for k in KEYS}
    return X1, I1


@pytest.mark.parametrize("kind,variant,resample", [("srht", "polyak", "fresh"),
                                                   ("srht", "gd", "nested"),
                                                   ("gaussian", "polyak", "nested")])
def test_persistent_equals_launches_fp64(rs, kind, variant, resample):
    p = config_c1()
    nus = [3e-4, 1e-3, 1e-2, 0.1, 1.0]
    same(rs, dev_padded(p.A, rs), torch.from_numpy(p.b).cuda(), nus, kind=kind,
         variant=variant, resample=resample, seed=3)


@pytest.mark.parametrize("check_every", [1, 4])
def test_persistent_equals_launches_ragged(rs, check_every):
    # ragged n and d; seven nu converge after different numbers of steps and levels
    p = make_problem(3000, 70, spectrum("poly", 70, 0.8), 1e-3, 0.1, 7, dtype=np.float64)
    same(rs, dev_padded(p.A, rs), torch.from_numpy(p.b).cuda(), list(np.logspace(-5, 0, 7)),
         seed=11, check_every=check_every)


@pytest.mark.parametrize("sketch_dtype", ["f32", "bf16"])
def test_persistent_equals_launches_fp32(rs, sketch_dtype):
    p = make_problem(16384, 256, spectrum("poly", 256, 0.8), 1e-3, 0.1, 5)
    nus = list(np.logspace(-6, 0, 16))
    X, infos = same(rs, dev_padded(p.A, rs), torch.from_numpy(p.b).cuda(), nus,
                    sketch_dtype=sketch_dtype)
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    G = A64.T @ A64
    Atb = A64.T @ b64
    Xh = host(X)
    for k in (0, 7, 15):
        xs = ridge.solve_direct_from_gram(G, Atb, nus[k])
        assert ridge.relative_error(G + nus[k] * np.eye(256), Xh[k], xs) <= 1e-6


def test_persistent_full_size(rs):
    # 2^18 x 2048, 64 nu^2 (Kc up to 128 columns): identical to the launches
    A0, b = make_c4a_problem("cuda")
    A = rs.padded(A0.shape[0], A0.shape[1], dtype=torch.float32)
    A.copy_(A0)
    del A0
    X, infos = same(rs, A, b, list(config_c4a_nu2()), sketch_dtype="bf16")
    assert all(i["status"] == "ok" for i in infos)
