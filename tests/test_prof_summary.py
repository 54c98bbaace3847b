"""Host logic of the profile summaries (no GPU): the per-level split of a
V-cycle from a synthetic kernel trace, the trace table and the counter
scaling of the HBM traffic record."""
import csv
import json

from paper_2504_00724_amd import prof_summary as P


def _trace(path, launches, gap0=1000000):
    """launches: [(name, duration_ns, gap_before_ns)] written as a kernel trace csv."""
    t = 0
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, d, gap in launches:
            t += gap
            w.writerow({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + d})
            t += d


def _fused(fin, pro, norm=False):
    return "void k_smooth_fused<double, false, %s, 16, %s, %s>(...)" % (
        "true" if fin else "false", "true" if pro else "false", "true" if norm else "false")


def _cycle(levels, nu=2, pipe=False):
    """A V-cycle on `levels` levels (0 finest): nu fused steps and a
    restriction per level going down, the coarsest solve, then nu fused
    steps per level going up (the first applying the correction), then the
    norm: a norm launch, or (pipe) the next cycle's first fused step, which
    takes it (that cycle then has one finest-level pre-step less)."""
    out = []
    for m in range(levels - 1):
        steps = nu - 1 if (pipe and m == 0) else nu
        out += [(_fused(m == 0, False), 1000 * (levels - m), 0)] * steps
        out.append(("void k_restrict<double, double, false, false>(...)", 500, 0))
    out.append(("void k_coarse<double>(...)", 700, 0))
    for m in range(levels - 2, -1, -1):
        out.append((_fused(m == 0, True), 1000 * (levels - m), 0))
        out += [(_fused(m == 0, False), 1000 * (levels - m), 0)] * (nu - 1)
    if pipe:
        out.append((_fused(True, False, norm=True), 1000 * levels, 0))
    else:
        out.append(("void k_resnorm<double, false>(...)", 300, 0))
    out.append(("__amd_rocclr_copyBuffer", 100, 50000))
    return out


def _split(tmp_path, capsys, pipe):
    path = tmp_path / "t_kernel_trace.csv"
    launches = [("k_gj_elim", 100, 0)] * 5                      # set-up, then an idle gap
    solve = [(_fused(True, False, norm=True), 4000, 0)] if pipe else []
    for _ in range(3):
        solve += _cycle(4, pipe=pipe)
    launches += [(n, d, g) for n, d, g in solve]
    launches[5] = (launches[5][0], launches[5][1], 400000)      # the solve starts after a long gap
    _trace(path, launches)

    class A:
        pass
    a = A()
    a.path = str(path)
    P.cmd_cycle(a)
    out = capsys.readouterr().out
    head, seq = out.split("The launches of that cycle in order")
    rows = {l.split("|")[1].strip(): l for l in head.splitlines() if l.startswith("| ")}
    rows["_seq"] = [[c.strip() for c in l.split("|")[1:-1]] for l in seq.splitlines() if l.startswith("| ") and
                    not l.startswith("| #") and not l.startswith("|---")]
    return rows


def test_cycle_split_by_level(tmp_path, capsys):
    rows = _split(tmp_path, capsys, False)
    # per level: 2 down + 2 up fused steps + 1 restriction (levels 0..2); level 3 is the coarsest
    for m in range(3):
        cells = [c.strip() for c in rows[str(m)].split("|")]
        assert cells[2] == "5"
        assert abs(float(cells[3]) - (4 * (4 - m) + 0.5)) < 1e-9
    assert "`k_coarse<double>`" in rows and "`k_resnorm<double, false>`" in rows


def test_cycle_split_when_the_first_step_takes_the_norm(tmp_path, capsys):
    """Cycles delimited by the norm-taking first fused step (no norm
    launch): the step counts on level 0 (it closes the cycle there)."""
    rows = _split(tmp_path, capsys, True)
    for m in range(3):
        cells = [c.strip() for c in rows[str(m)].split("|")]
        assert cells[2] == "5"
        assert abs(float(cells[3]) - (4 * (4 - m) + 0.5)) < 1e-9
    assert "`k_coarse<double>`" in rows and not any("k_resnorm" in k for k in rows)


def test_cycle_launch_sequence(tmp_path, capsys):
    """The per-launch table lists every launch of the cycle once, in order,
    with the level the descent and ascent assign to it."""
    rows = _split(tmp_path, capsys, True)
    seq = rows["_seq"]
    other = [k for k in rows if k.startswith("`")]                              # coarsest solve, copies
    nlaunch = sum(int(rows[str(m)].split("|")[2]) for m in range(3)) + len(other)
    assert len(seq) == nlaunch
    assert [int(r[0]) for r in seq] == list(range(1, nlaunch + 1))
    levels = [r[1] for r in seq]
    assert levels[-1] == "0"
    ic = [r[2] for r in seq].index("`k_coarse<double>`")
    assert levels[ic] == ""
    down = [v for v in levels[:ic] if v]
    assert down == sorted(down, key=int)                                         # the descent only goes down


def test_traffic_record_scaling(tmp_path, capsys):
    def counters(path, counter, vals):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for k, v in vals:
                w.writerow({"Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})
    cells = 1024
    known = 8.0 * cells / 1024.0                                  # KiB the copy reads and writes
    counters(tmp_path / "f.csv", "FETCH_SIZE", [("k_copy", known / 2), ("k_x", 10.0), ("k_y", 4.0)])
    counters(tmp_path / "w.csv", "WRITE_SIZE", [("k_copy", known), ("k_x", 3.0), ("k_y", 1.0)])

    class A:
        pass
    a = A()
    a.fetch, a.write, a.cells, a.kernel, a.calib_kernel = str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), cells, \
        ["k_x", "k_y"], "k_copy"
    P.cmd_pmc(a)
    out = capsys.readouterr().out
    rec = json.loads(out.split("<!-- traffic-record ")[1].rsplit("-->", 1)[0])
    assert rec["kernel"] == "k_x"
    assert abs(rec["scale_fetch"] - 2.0) < 1e-12 and abs(rec["scale_write"] - 1.0) < 1e-12
    assert abs(rec["traffic_bytes_per_launch"] - (10.0 * 2.0 + 3.0) * 1024.0) < 1e-9
    # one record per kernel; the lookup picks the named one
    md = tmp_path / "p.md"
    md.write_text(out)
    ry = P.read_traffic_record(str(md), "k_y")
    assert ry["kernel"] == "k_y" and abs(ry["traffic_bytes_per_launch"] - (4.0 * 2.0 + 1.0) * 1024.0) < 1e-9
    assert P.read_traffic_record(str(md), "k_z") is None
