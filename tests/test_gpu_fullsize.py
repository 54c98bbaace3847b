"""Parity at the benchmark's full size (three-circle Poisson workload at
2048^2, default options as the benchmark runs them), through the C ABI.

The oracle builds the full cut-cell geometry and classification at 2048^2
and fits the least-squares rows of all irregular cells (29 K rows, fitted in
worker processes, tests/oracle_jobs.py).  Checked against it:

* cell kinds and merge hosts on every cell (bit-exact);
* the lattice of every irregular row (bit-exact) and its weights;
* the GPU operator on every non-empty cell for a random u;
* the converged GPU solution through its residual f - N g - L u on every
  non-empty cell, recomputed here in FP64 (difference form) from the
  oracle's rows (the solve reached 1e-10 of the system the oracle
  assembles), and its error against the manufactured solution;
* mixed precision against FP64 at the same size (within the
  discretization error).
"""
import numpy as np
import pytest

import oracle_jobs
import workloads as W
from oracle.discretization import Discretization, regular_coefficients
from oracle.geometry import CutGrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 2048


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_00724_amd.ccgmg import Solver
    import bench
    dev = torch.device("cuda:0")
    cfg = W.config(4, n=N)
    print("full-size parity: building the library context (2048^2)", flush=True)
    S = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], tol=1e-10, max_cycles=200,
               hip_stream=torch.cuda.current_stream().cuda_stream)
    f, g, exact, kinds = bench.make_inputs(S, cfg, torch, dev)
    print("full-size parity: oracle geometry (2048^2)", flush=True)
    cg = CutGrid(cfg["grid"], cfg["curves"])
    d = Discretization(cg, cfg["a"], cfg["b"], cfg["c"], eager=False)
    print("full-size parity: fitting all %d oracle rows in worker processes" % len(d.irregular), flush=True)
    rows = oracle_jobs.all_rows(4, N, d.irregular)
    irr = np.asarray(d.irregular)
    R = dict(cells=np.array([rows[int(q)][0] for q in irr], dtype=np.int64),
             w=np.array([rows[int(q)][1] for q in irr]),
             fq=np.array([k for k, q in enumerate(irr) for _ in rows[int(q)][2]], dtype=np.int64),
             ff=np.array([fk for q in irr for fk, _ in rows[int(q)][2]], dtype=np.int64),
             fw=np.array([wf for q in irr for _, wf in rows[int(q)][2]]))
    print("full-size parity: oracle rows ready", flush=True)
    yield dict(S=S, cfg=cfg, cg=cg, d=d, f=f, g=g, exact=exact, kinds=kinds, rows=rows, R=R, irr=irr, dev=dev)
    S.close()


def _oracle_apply(F, u):
    """(L u) on every non-empty cell from the oracle's regular stencil and
    rows, in difference form, and |L||u| row by row."""
    d, R, irr = F["d"], F["R"], F["irr"]
    nx = ny = N
    U = u.reshape(ny, nx)
    P = np.zeros((ny + 4, nx + 4))
    P[2:-2, 2:-2] = U
    A = np.abs(P)
    acc = np.zeros((ny, nx))
    mag = np.zeros((ny, nx))
    coef = regular_coefficients(d.a, d.b, d.c, d.h)
    for (dx, dy), v in coef.items():
        sl = (slice(2 + dy, 2 + dy + ny), slice(2 + dx, 2 + dx + nx))
        if (dx, dy) != (0, 0):
            acc += v * (P[sl] - U)
        mag += abs(v) * A[sl]
    acc += sum(coef.values()) * U
    out = np.where(d.regular.reshape(ny, nx), acc, 0.0).ravel()
    mag = np.where(d.regular.reshape(ny, nx), mag, 0.0).ravel()
    uq = u[irr][:, None]
    out[irr] = np.sum(R["w"] * (u[R["cells"]] - uq), axis=1) + R["w"].sum(axis=1) * u[irr]
    mag[irr] = np.sum(np.abs(R["w"]) * np.abs(u[R["cells"]]), axis=1)
    return out, mag


def test_fullsize_classification_and_all_rows(full):
    S, d, cg = full["S"], full["d"], full["cg"]
    kind, host = S.kinds(0)
    assert np.array_equal(kind, d.kind)
    assert np.array_equal(host, cg.host)
    rows, cols, vals, _ = S.irregular(0)
    assert np.array_equal(rows, d.irregular)
    fcell, fcurve, nweight = S.boundary_faces()
    assert [(int(a), int(b)) for a, b in zip(fcell, fcurve)] == d.faces
    R = full["R"]
    assert np.array_equal(cols, R["cells"])
    werr = np.max(np.abs(vals - R["w"])) * d.h ** 2
    ref_nw = np.zeros(len(d.faces))
    ref_nw[R["ff"]] = R["fw"]
    # Dirichlet data everywhere: boundary weights in 1/h^2 units like the cells'
    nerr = np.max(np.abs(nweight - ref_nw)) * d.h ** 2
    print("full-size rows: %d lattices equal, weight error %.2e, boundary weight error %.2e (h^2 units)"
          % (len(rows), werr, nerr), flush=True)
    assert werr <= 1e-12
    assert nerr <= 1e-12


def test_fullsize_operator_on_every_cell(full):
    S, d, dev = full["S"], full["d"], full["dev"]
    rng = np.random.default_rng(7)
    u = rng.standard_normal(N * N) * d.nonempty
    out = torch.zeros(N * N, dtype=torch.float64, device=dev)
    S.apply(torch.tensor(u, device=dev), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref, mag = _oracle_apply(full, u)
    ne = d.nonempty
    worst = np.max(np.abs(got - ref)[ne] / mag[ne])
    print("full-size operator: worst |L u - oracle| / (|L||u|) = %.2e over %d cells" % (worst, int(ne.sum())),
          flush=True)
    assert worst <= 1e-12
    assert np.all(got[~ne] == 0.0)


def test_fullsize_solution_residual_and_error(full):
    S, d, dev, R, irr = full["S"], full["d"], full["dev"], full["R"], full["irr"]
    f, g = full["f"], full["g"]
    S.set_boundary(g, 1)
    u = torch.zeros_like(f)
    rep = S.solve(f, u)
    torch.cuda.synchronize()
    uh = u.cpu().numpy()
    rhs = f.cpu().numpy().copy()
    gh = g.cpu().numpy()
    # f - N g on every non-empty cell (N from the oracle's rows)
    np.subtract.at(rhs, irr[R["fq"]], R["fw"] * gh[R["ff"]])
    Lu, _ = _oracle_apply(full, uh)
    ne = d.nonempty
    rel = np.max(np.abs(rhs - Lu)[ne]) / np.max(np.abs(rhs)[ne])
    err = np.max(np.abs(uh - full["exact"])[ne])
    print("full-size solve: cycles %d, library rel_res %.2e, oracle residual on every cell %.2e, error vs exact %.2e"
          % (rep["cycles"], rep["rel_res_inf"], rel, err), flush=True)
    assert rep["rel_res_inf"] <= 1e-10
    assert rel <= 1.5e-10
    assert err < 1e-8          # fourth order: ~3e-9 at h = 1/2048 for this workload
    assert np.all(uh[~ne] == 0.0)
    full["u64"] = uh


def test_fullsize_mixed_precision_matches_fp64(full):
    from paper_2504_00724_amd.ccgmg import Solver
    if "u64" not in full:
        pytest.skip("needs the FP64 solve")
    cfg, dev = full["cfg"], full["dev"]
    Sm = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], tol=1e-10, max_cycles=200,
                hip_stream=torch.cuda.current_stream().cuda_stream, precision=1)
    Sm.set_boundary(full["g"], 1)
    u = torch.zeros_like(full["f"])
    rep = Sm.solve(full["f"], u)
    torch.cuda.synchronize()
    um = u.cpu().numpy()
    ne = full["d"].nonempty
    diff = np.max(np.abs(um - full["u64"])[ne])
    disc = np.max(np.abs(full["u64"] - full["exact"])[ne])
    print("mixed precision at 2048^2: cycles %d rel_res %.2e, |u_mp - u_fp64| %.2e, discretization error %.2e"
          % (rep["cycles"], rep["rel_res_inf"], diff, disc), flush=True)
    assert rep["rel_res_inf"] <= 1e-10
    assert diff <= disc
    Sm.close()


def test_fullsize_adjoint_gradients_match_finite_differences(full):
    """The adjoint workload at 2048^2: J = 1/2 ||u - u_target||^2 over the
    non-empty cells, u_target = <u> + N(0, 1e-3^2) (seed 44); gradients with
    respect to f-hat and g-hat from the autograd Function (adjoint solve on
    L^T, then -N^T lambda) against central differences along 16 unit
    directions in (f-hat, g-hat) (seeds 400-415: smooth 4 x 4-mode Fourier
    fields on the cells, N(0,1) on the boundary faces).  J is quadratic in
    the data, so the central difference is exact for any eps; it is
    evaluated as 1/2 sum (u+ - u-)(u+ + u- - 2 u_target) to avoid cancelling
    two large values of J, and both solves of a pair must take the same
    number of cycles (then both are the same linear map, which differs from
    L^{-1} by the ~1e-9 error operator of that many cycles).  eps = 1e-2:
    with eps = 1e-6 the perturbation of u (~5e-11 per cell) is at the
    rounding level of the solves themselves (~1e-13 per cell after the sum
    over 3.8 M cells) and the comparison only shows that noise."""
    from paper_2504_00724_amd.autograd import cutcell_solve
    S, d, dev = full["S"], full["d"], full["dev"]
    f, g = full["f"], full["g"]
    mask_np = d.nonempty.astype(np.float64)
    mask = torch.tensor(mask_np, device=dev)
    target = torch.tensor((full["exact"] + 1e-3 * np.random.default_rng(44).standard_normal(N * N)) * mask_np,
                          device=dev)
    fr = f.clone().requires_grad_(True)
    gr = g.clone().requires_grad_(True)
    u = cutcell_solve(fr, gr, S)
    J = 0.5 * torch.sum(((u - target) * mask) ** 2)
    J.backward()
    gf, gg = fr.grad.detach(), gr.grad.detach()
    gnorm = float(torch.sqrt(torch.sum(gf ** 2) + torch.sum(gg ** 2)))   # bounds |dJ . d| for unit d
    h = 1.0 / N
    xc = (np.arange(N) + 0.5) * h
    eps = 1e-2
    worst = 0.0
    for k in range(16):
        rng = np.random.default_rng(400 + k)
        c = rng.standard_normal((4, 4))
        sx = np.sin(np.pi * np.outer(np.arange(1, 5), xc))           # [p][i]
        df = (sx.T @ c.T @ sx).ravel() * mask_np                       # [j][i]
        dg = rng.standard_normal(g.numel())
        nrm = np.sqrt(np.sum(df ** 2) + np.sum(dg ** 2))
        df_t, dg_t = torch.tensor(df / nrm, device=dev), torch.tensor(dg / nrm, device=dev)
        up, um = torch.zeros_like(f), torch.zeros_like(f)
        S.set_boundary(g + eps * dg_t, 1)
        rp = S.solve(f + eps * df_t, up)
        S.set_boundary(g - eps * dg_t, 1)
        rm = S.solve(f - eps * df_t, um)
        assert rp["cycles"] == rm["cycles"]
        fd = float(0.5 * torch.sum((up - um) * (up + um - 2.0 * target) * mask ** 2)) / (2.0 * eps)
        adj = float(torch.sum(gf * df_t) + torch.sum(gg * dg_t))
        rel = abs(fd - adj) / gnorm
        worst = max(worst, rel)
        print("   direction %2d: fd %.10e adjoint %.10e |fd - adjoint| / |grad J| %.2e" % (k, fd, adj, rel),
              flush=True)
    S.set_boundary(g, 1)
    # error relative to |grad J| (the largest directional derivative over
    # unit directions): directions nearly orthogonal to grad J would
    # otherwise divide the solve's rounding floor by a tiny number
    assert worst < 1e-8
