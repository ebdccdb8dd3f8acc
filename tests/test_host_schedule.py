"""Host-side checks of the level schedules the symbolic pass builds (no GPU).

``tests/native/schedule_check.cpp`` replays the order in which the kernels
run the factorisation and the triangular solves (one barrier-separated pass
per metadata chunk, one wavefront's lanes per row) and checks that every
value is read after the pass that last writes it, that the lanes of one task
are ordered where they share values, that chunks break on level boundaries,
and that the adjoint's transposed schedules mirror the forward ones.  It is
built here with AddressSanitizer and UndefinedBehaviorSanitizer together
with the library's host modules (symbolic analysis and operator patterns),
so the sanitizers cover those modules on every grid.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from gen.grids import SPECS, make_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_07099_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("schedule") / "schedule_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "native", "schedule_check.cpp"), os.path.join(CSRC, "symbolic.cpp"),
           os.path.join(CSRC, "operators.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return out


def _write_net(path, n_bus, bus_type, f, t, r, x, bc):
    with open(path, "w") as fh:
        fh.write(f"{n_bus} {len(f)}\n" + " ".join(str(int(v)) for v in bus_type) + "\n")
        for k in range(len(f)):
            fh.write("%d %d %.17g %.17g %.17g\n" % (f[k], t[k], r[k], x[k], bc[k]))


def _run(checker, path, *opts):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([checker, path, *opts], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "violations 0" in r.stdout, r.stdout
    return r.stdout


@pytest.mark.parametrize("name", list(SPECS))
def test_schedules_are_ordered_on_every_grid(checker, tmp_path, name):
    spec, net, sc = make_case(name, batch=1)
    p = str(tmp_path / f"{name}.txt")
    _write_net(p, net.n_bus, net.bus_type, net.f, net.t, net.r, net.x, net.bc)
    # the dense tail of FP32 (32 rows) and FP64 (16 rows) templates; the
    # largest metadata chunk and a small one that splits levels over chunks
    for tail in ("32", "16"):
        for budget in ("12288", "320"):
            out = _run(checker, p, "--tail", tail, "--budget", budget)
            assert "intra_task_hazards 0" in out


def test_edge_networks(checker, tmp_path):
    """A path (every level one row), a star around the slack (one level) and
    a two-bus network."""
    rng = np.random.default_rng(3)
    cases = []
    n = 40
    cases.append((n, [2] + [0] * (n - 1), list(range(n - 1)), list(range(1, n))))
    cases.append((n, [2] + [1, 0] * ((n - 1) // 2) + [0] * ((n - 1) % 2), [0] * (n - 1), list(range(1, n))))
    cases.append((2, [2, 0], [0], [1]))
    for i, (nb, bt, f, t) in enumerate(cases):
        m = len(f)
        r = rng.uniform(0.005, 0.05, m)
        p = str(tmp_path / f"edge{i}.txt")
        _write_net(p, nb, bt, f, t, r, 5 * r, np.zeros(m))
        for tail in ("32", "0"):
            _run(checker, p, "--tail", tail, "--budget", "320")


def test_replay_of_fill_side_pivot_inversion_is_ordered(checker, tmp_path):
    """The variant that inverts the pivot blocks of rows without L blocks in
    the Jacobian fill (before the fill's closing barrier) and starts the
    factorisation one level later: its reads of those inverses all follow the
    barrier, so ordering across passes does not explain the non-finite
    iterates it gave on the 1354-bus batch."""
    for name in ("c2", "c4"):
        spec, net, sc = make_case(name, batch=1)
        p = str(tmp_path / f"{name}.txt")
        _write_net(p, net.n_bus, net.bus_type, net.f, net.t, net.r, net.x, net.bc)
        _run(checker, p, "--variant-fill-inverts-level0")
