"""GPU parity of the HIP solver against the oracle, through the C-ABI."""
import numpy as np
import pytest

import workloads as W
from oracle.discretization import boundary_data
from oracle.geometry import cell_averages
from oracle.multigrid import Level, direct_solve, rhs_vector

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [(1, 64), (2, 64), (4, 128), (5, 64)]
_LEVELS = {}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _level(k, n):
    if (k, n) not in _LEVELS:
        cfg = W.config(k, n=n)
        lv = Level(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
        _LEVELS[(k, n)] = (cfg, lv)
    return _LEVELS[(k, n)]


def _solver(cfg, **kw):
    from paper_2504_00724_amd.ccgmg import Solver
    return Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"],
                  hip_stream=torch.cuda.current_stream().cuda_stream, **kw)


@pytest.mark.parametrize("k,n", CASES)
def test_apply_matches_oracle(k, n):
    dev = _dev()
    cfg, lv = _level(k, n)
    print("apply parity config %d n=%d" % (k, n), flush=True)
    S = _solver(cfg)
    rng = np.random.default_rng(10 + k)
    absL = abs(lv.L)
    for u in (rng.standard_normal(n * n) * lv.nonempty, cell_averages(lv.cg, cfg["solution"].u).ravel()):
        ud = torch.tensor(u, device=dev)
        out = torch.zeros_like(ud)
        S.apply(ud, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = lv.L @ u
        scale = absL @ np.abs(u)
        ne = lv.nonempty
        assert np.all(np.abs(got - ref)[ne] <= 1e-12 * scale[ne] + 1e-300)
        assert np.all(got[~ne] == 0.0)
    S.close()


@pytest.mark.parametrize("k,n", CASES)
def test_solve_matches_oracle_direct(k, n):
    dev = _dev()
    cfg, lv = _level(k, n)
    print("solve parity config %d n=%d" % (k, n), flush=True)
    f = cell_averages(lv.cg, cfg["f"]).ravel()
    g = boundary_data(lv.disc, cfg["solution"])
    ref = direct_solve(lv, rhs_vector(lv, f, g))
    S = _solver(cfg, tol=1e-12, max_cycles=200)
    fd = torch.tensor(f, device=dev)
    S.set_boundary(torch.tensor(g, device=dev), 1)
    u = torch.zeros_like(fd)
    rep = S.solve(fd, u)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print("   cycles %d rel_res %.2e rel_err %.2e levels %d" % (rep["cycles"], rep["rel_res_inf"], err,
                                                               S.info["n_levels"]), flush=True)
    assert err <= 1e-10
    assert np.all(got[~lv.nonempty] == 0.0)
    S.close()


def test_mixed_precision_within_discretization_error():
    dev = _dev()
    cfg, lv = _level(4, 128)
    f = cell_averages(lv.cg, cfg["f"]).ravel()
    g = boundary_data(lv.disc, cfg["solution"])
    ref = direct_solve(lv, rhs_vector(lv, f, g))
    exact = cell_averages(lv.cg, cfg["solution"].u).ravel()
    disc_err = np.max(np.abs(ref - exact)[lv.nonempty])
    S = _solver(cfg, tol=1e-10, precision=1)
    fd = torch.tensor(f, device=dev)
    S.set_boundary(torch.tensor(g, device=dev), 1)
    u = torch.zeros_like(fd)
    rep = S.solve(fd, u)
    torch.cuda.synchronize()
    err = np.max(np.abs(u.cpu().numpy() - ref)[lv.nonempty])
    print("mixed precision: cycles %d rel_res %.2e err vs oracle %.2e (disc err %.2e)" % (
        rep["cycles"], rep["rel_res_inf"], err, disc_err), flush=True)
    assert rep["rel_res_inf"] <= 1e-10
    assert err <= disc_err
    S.close()


def test_batched_right_hand_sides():
    dev = _dev()
    cfg, lv = _level(1, 64)
    rng = np.random.default_rng(7)
    F = np.stack([rng.standard_normal(64 * 64) * lv.nonempty for _ in range(3)])
    S = _solver(cfg, tol=1e-11, max_nrhs=3)
    fd = torch.tensor(F, device=dev)
    u = torch.zeros_like(fd)
    S.solve(fd, u, nrhs=3)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    for z in range(3):
        ref = direct_solve(lv, F[z])
        assert np.max(np.abs(got[z] - ref)) <= 1e-10 * np.max(np.abs(ref))
    S.close()
