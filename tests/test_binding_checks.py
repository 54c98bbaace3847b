"""Argument checks of the Python binding and the autograd wrapper (CPU).

The binding hands raw device pointers to the library, so it must refuse
anything that is not a contiguous float64 GPU tensor of the expected size
before the library sees it.  GPU tensors are imitated here by a CPU tensor
whose ``is_cuda`` reads True: the checks run, the library is never called.
"""
import numpy as np
import pytest

import workloads as W
from paper_2504_00724_amd import ccgmg

torch = pytest.importorskip("torch")


class _FakeGpu(torch.Tensor):
    @property
    def is_cuda(self):
        return True


def _fake(t):
    return torch.Tensor._make_subclass(_FakeGpu, t)


def _host_solver():
    try:
        ccgmg.lib()
    except RuntimeError:
        pytest.skip("libccgmg.so not built")
    return ccgmg.Solver(W.grid(16), [W.box(), W.circle(0.5, 0.5, 0.2)], 1.0, 0.0, 1.0, host_only=1)


def test_dev_pointer_checks():
    n = 256
    with pytest.raises(ValueError, match="torch tensor"):
        ccgmg._dev(np.zeros(n), n, "f")
    with pytest.raises(ValueError, match="GPU"):
        ccgmg._dev(torch.zeros(n, dtype=torch.float64), n, "f")
    with pytest.raises(ValueError, match="float64"):
        ccgmg._dev(_fake(torch.zeros(n, dtype=torch.float32)), n, "f")
    with pytest.raises(ValueError, match="contiguous"):
        ccgmg._dev(_fake(torch.zeros(2 * n, dtype=torch.float64)[::2]), n, "f")
    with pytest.raises(ValueError, match="elements"):
        ccgmg._dev(_fake(torch.zeros(n - 1, dtype=torch.float64)), n, "f")
    t = _fake(torch.zeros(n, dtype=torch.float64))
    assert ccgmg._dev(t, n, "f") == t.data_ptr()
    for bad in (0, -1, 1.5, "2"):
        with pytest.raises(ValueError):
            ccgmg._count(bad)


def test_solver_refuses_bad_arrays_before_the_library():
    S = _host_solver()
    n = S.n_cells
    nf = S.info["n_bdry_faces"]
    assert nf > 0
    good = _fake(torch.zeros(n, dtype=torch.float64))
    cpu = torch.zeros(n, dtype=torch.float64)
    with pytest.raises(ValueError):
        S.solve(cpu, good)
    with pytest.raises(ValueError):
        S.solve(good, _fake(torch.zeros(n, dtype=torch.float32)))
    # nrhs planes are required of f and u
    with pytest.raises(ValueError, match="elements"):
        S.solve(good, good, nrhs=2)
    with pytest.raises(ValueError, match="elements"):
        S.residual_norms(good, good, nrhs=3)
    # boundary data: n_faces per right-hand side
    with pytest.raises(ValueError, match="elements"):
        S.set_boundary(_fake(torch.zeros(nf, dtype=torch.float64)), 2)
    with pytest.raises(ValueError, match="elements"):
        S.apply_NT(good, _fake(torch.zeros(nf + 1, dtype=torch.float64)))
    with pytest.raises(ValueError, match="elements"):
        S.apply(good, _fake(torch.zeros(n + 16, dtype=torch.float64)))
    with pytest.raises(ValueError):
        S.tune(cpu)
    S.close()


class _StubSolver:
    """Stands in for Solver: u = f - B g per plane (B a fixed face-to-cell
    matrix), the adjoint lambda = rhs, N^T lambda = B^T lambda -- a linear
    map whose gradients are known in closed form."""

    def __init__(self, n, nf, seed=0):
        self.n_cells = n
        self.info = {"n_bdry_faces": nf}
        self.B = torch.tensor(np.random.default_rng(seed).standard_normal((n, nf)))
        self.g = None
        self.calls = []

    def set_boundary(self, g, nrhs):
        assert g.is_contiguous() and g.numel() == nrhs * self.info["n_bdry_faces"]
        self.g = g.reshape(nrhs, -1).clone()
        self.calls.append(("set_boundary", nrhs))

    def solve(self, f, u, nrhs):
        assert f.numel() == u.numel() == nrhs * self.n_cells
        u.copy_((f.reshape(nrhs, -1) - self.g @ self.B.T).reshape(u.shape))

    def solve_adjoint(self, rhs, lam, nrhs):
        assert rhs.numel() == lam.numel() == nrhs * self.n_cells
        lam.copy_(rhs)

    def apply_NT(self, lam, out, nrhs):
        assert out.numel() == nrhs * self.info["n_bdry_faces"]
        out.copy_(lam.reshape(nrhs, -1) @ self.B)


@pytest.mark.parametrize("nrhs,shared", [(1, True), (3, True), (3, False)])
def test_autograd_boundary_shapes(nrhs, shared):
    from paper_2504_00724_amd.autograd import cutcell_solve
    n, nf = 20, 6
    S = _StubSolver(n, nf)
    rng = np.random.default_rng(1)
    f = torch.tensor(rng.standard_normal((nrhs, n)) if nrhs > 1 else rng.standard_normal(n), requires_grad=True)
    g = torch.tensor(rng.standard_normal(nf) if shared else rng.standard_normal((nrhs, nf)), requires_grad=True)
    u = cutcell_solve(f, g, S)
    assert u.shape == f.shape
    w = torch.tensor(rng.standard_normal(tuple(u.shape)))
    (u * w).sum().backward()
    # J = sum w (f - B g): dJ/df = w, dJ/dg = -B^T w (summed over planes when g is shared)
    assert torch.allclose(f.grad, w)
    wg = w.reshape(nrhs, n) @ S.B
    ref = -wg.sum(dim=0) if (shared and nrhs > 1) else -wg.reshape(g.shape)
    assert g.grad.shape == g.shape
    assert torch.allclose(g.grad, ref)


def test_autograd_rejects_mismatched_shapes():
    from paper_2504_00724_amd.autograd import cutcell_solve
    S = _StubSolver(20, 6)
    with pytest.raises(ValueError):
        cutcell_solve(torch.zeros(3, 20, dtype=torch.float64), torch.zeros(2, 6, dtype=torch.float64), S)
    with pytest.raises(ValueError):
        cutcell_solve(torch.zeros(3, 20, dtype=torch.float64), torch.zeros(5, dtype=torch.float64), S)
    with pytest.raises(ValueError):
        cutcell_solve(torch.zeros(3, 21, dtype=torch.float64), torch.zeros(6, dtype=torch.float64), S)
