"""Parity at the benchmark's full size (three-circle Poisson workload at
2048^2, default options as the benchmark runs them), through the C ABI.

The oracle builds the full cut-cell geometry and classification at 2048^2
and fits least-squares rows for a seeded sample of irregular cells only
(fitting all 29 K rows takes minutes).  Checked against it:

* cell kinds and merge hosts on every cell (bit-exact);
* lattices (bit-exact) and weights of the sampled rows;
* the GPU operator on sampled rows (irregular and regular) for a random u;
* the converged GPU solution through its residual on sampled rows,
  recomputed here in FP64 from the oracle's rows (a property that holds at
  any size: the solve reached 1e-10 of the system the oracle assembles),
  and its error against the manufactured solution;
* mixed precision against FP64 at the same size (within the
  discretization error).
"""
import numpy as np
import pytest

import workloads as W
from oracle.discretization import Discretization, regular_coefficients
from oracle.geometry import CutGrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 2048
SAMPLES = 96


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
    rng = np.random.default_rng(2048)
    sample = np.sort(rng.choice(d.irregular, size=SAMPLES, replace=False))
    print("full-size parity: fitting %d sampled oracle rows" % SAMPLES, flush=True)
    rows = {int(q): d.row(int(q)) for q in sample}
    yield dict(S=S, cfg=cfg, cg=cg, d=d, f=f, g=g, exact=exact, kinds=kinds, sample=sample, rows=rows, dev=dev)
    S.close()


def _oracle_Lu(F, q, u):
    """(L u)_q from the oracle's row (difference form) and |L||u| at q."""
    d = F["d"]
    nx = d.nx
    if d.regular[q]:
        coef = regular_coefficients(d.a, d.b, d.c, d.h)
        i, j = q % nx, q // nx
        acc, mag = 0.0, 0.0
        for (dx, dy), w in coef.items():
            k = (j + dy) * nx + i + dx
            if (dx, dy) != (0, 0):
                acc += w * (u[k] - u[q])
            mag += abs(w) * abs(u[k])
        return acc + sum(coef.values()) * u[q], mag
    cells, w, _ = F["rows"][q]
    acc = sum(wk * (u[k] - u[q]) for k, wk in zip(cells, w)) + float(np.sum(w)) * u[q]
    return acc, float(np.sum(np.abs(w) * np.abs(u[np.array(cells)])))


def test_fullsize_classification_and_sampled_rows(full):
    S, d, cg = full["S"], full["d"], full["cg"]
    kind, host = S.kinds(0)
    assert np.array_equal(kind, d.kind)
    assert np.array_equal(host, cg.host)
    rows, cols, vals, _ = S.irregular(0)
    assert np.array_equal(rows, d.irregular)
    fcell, fcurve, _ = S.boundary_faces()
    assert [(int(a), int(b)) for a, b in zip(fcell, fcurve)] == d.faces
    pos = {int(q): i for i, q in enumerate(rows)}
    for q in full["sample"]:
        q = int(q)
        cells, w, _ = full["rows"][q]
        i = pos[q]
        assert list(cols[i]) == list(cells)
        assert np.max(np.abs(vals[i] - w)) * d.h ** 2 <= 1e-12


def test_fullsize_operator_on_sampled_rows(full):
    S, d, dev = full["S"], full["d"], full["dev"]
    rng = np.random.default_rng(7)
    u = rng.standard_normal(N * N) * d.nonempty
    out = torch.zeros(N * N, dtype=torch.float64, device=dev)
    S.apply(torch.tensor(u, device=dev), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    regular = np.flatnonzero(d.regular)
    reg_sample = rng.choice(regular, size=SAMPLES, replace=False)
    for q in list(full["sample"]) + list(reg_sample):
        ref, mag = _oracle_Lu(full, int(q), u)
        assert abs(got[q] - ref) <= 1e-12 * mag, (int(q), got[q], ref)


def test_fullsize_solution_residual_and_error(full):
    S, d, dev = full["S"], full["d"], full["dev"]
    f, g = full["f"], full["g"]
    S.set_boundary(g, 1)
    u = torch.zeros_like(f)
    rep = S.solve(f, u)
    torch.cuda.synchronize()
    uh = u.cpu().numpy()
    fh = f.cpu().numpy()
    gh = g.cpu().numpy()
    # conservative reference norm: |f| on regular cells and |f - N g| on the
    # sampled irregular rows (a subset of the true max)
    ref = np.max(np.abs(fh[d.regular]))
    worst = 0.0
    rng = np.random.default_rng(11)
    reg_sample = rng.choice(np.flatnonzero(d.regular), size=SAMPLES, replace=False)
    for q in list(full["sample"]) + list(reg_sample):
        q = int(q)
        Lu, _ = _oracle_Lu(full, q, uh)
        rhs = fh[q]
        if not d.regular[q]:
            for fk, wf in full["rows"][q][2]:
                rhs -= wf * gh[fk]
            ref = max(ref, abs(rhs))
        worst = max(worst, abs(rhs - Lu))
    rel = worst / ref
    err = np.max(np.abs(uh - full["exact"])[d.nonempty])
    print("full-size solve: cycles %d, library rel_res %.2e, sampled oracle residual %.2e, error vs exact %.2e"
          % (rep["cycles"], rep["rel_res_inf"], rel, err), flush=True)
    assert rep["rel_res_inf"] <= 1e-10
    assert rel <= 1.5e-10
    assert err < 1e-8          # fourth order: ~3e-9 at h = 1/2048 for this workload
    assert np.all(uh[~d.nonempty] == 0.0)
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
