"""The algorithmic FLOP count used for the roofline, counted mechanically.

tests/flopcount/ holds a counting scalar (flop.h) and a plain Carter-form
reference of the per-unit arithmetic (hotpath_ref.h).  The reference's
right-hand side and constraint diagnostics are checked here against the
oracle (so the counted computation is the method's), and its per-unit
counts must equal the constants bench.py prices a launch with.  The oracle
itself, compiled with the counting scalar for double, is counted too: its
matrix-inverse form of Hamilton's equations costs about 400 FLOP per
evaluation, over three times the Carter form's, so it overcounts what the
method needs and is not the basis."""
import json
import math
import os
import subprocess

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "flopcount", "flop_count.cpp")


@pytest.fixture(scope="module")
def counter(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("flop") / "flop_count")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fno-fast-math", "-ffp-contract=off", "-w", "-o", exe, SRC, "-lm"],
                   check=True)
    return exe


def test_reference_rhs_is_the_method(counter):
    """The counted Carter-form right-hand side, H and |H|_rel equal the
    oracle's (matrix inverse of eq:Kerr) at random states."""
    rng = np.random.default_rng(53)
    for _ in range(30):
        a = float(rng.uniform(-0.99, 0.99))
        E, L = float(rng.uniform(0.5, 1.5)), float(rng.uniform(-5, 5))
        r, th = float(rng.uniform(2.5, 500.0)), float(rng.uniform(0.2, 2.9))
        pr, pth = float(rng.uniform(-2, 2)), float(rng.uniform(-4, 4))
        out = subprocess.run([counter, "rhs", repr(a), repr(E), repr(L), repr(r), repr(th), repr(pr), repr(pth)],
                             capture_output=True, text=True, check=True).stdout.split()
        got = np.array([float(v) for v in out])
        z = np.array([r, th, 0.0, pr, pth])
        want = O.rhs(1.0, a, z, E, L)[:5]
        scale = np.abs(want).max()
        np.testing.assert_allclose(got[:5], want, rtol=1e-11, atol=1e-13 * scale)
        assert got[5] == pytest.approx(O.hamiltonian(1.0, a, z, E, L), rel=1e-10, abs=1e-13 * scale)
        assert got[6] == pytest.approx(O.hamiltonian_rel(1.0, a, z, E, L), rel=1e-9, abs=1e-14)


def test_reference_qmetric_rhs_is_the_method(counter):
    """The counted q-metric right-hand side and diagnostics equal the
    oracle's at random states."""
    rng = np.random.default_rng(75)
    for _ in range(20):
        q = float(rng.uniform(-0.4, 1.5))
        E, L = float(rng.uniform(0.5, 1.5)), float(rng.uniform(-5, 5))
        r, th = float(rng.uniform(2.5, 500.0)), float(rng.uniform(0.2, 2.9))
        pr, pth = float(rng.uniform(-2, 2)), float(rng.uniform(-4, 4))
        out = subprocess.run([counter, "qrhs", repr(q), repr(E), repr(L), repr(r), repr(th), repr(pr), repr(pth)],
                             capture_output=True, text=True, check=True).stdout.split()
        got = np.array([float(v) for v in out])
        z = np.array([r, th, 0.0, pr, pth])
        want = O.rhs_k(O.QMETRIC, 1.0, 0.0, q, z, E, L)[:5]
        np.testing.assert_allclose(got[:5], want, rtol=1e-10, atol=1e-13 * np.abs(want).max())
        assert got[5] == pytest.approx(O.hamiltonian_k(O.QMETRIC, 1.0, 0.0, q, z, E, L), rel=1e-10, abs=1e-13)
        assert got[6] == pytest.approx(O.hamiltonian_rel_k(O.QMETRIC, 1.0, 0.0, q, z, E, L), rel=1e-9, abs=1e-14)


def test_unit_counts_are_the_benchmark_basis(counter):
    import bench
    units = json.loads(subprocess.run([counter, "units"], capture_output=True, text=True, check=True).stdout)
    assert units == bench.FLOP_UNITS
    # Dormand-Prince: 26 nonzero stage coefficients and 6 error weights, times
    # 5 components, as multiply-adds (2 FLOP), plus the step's h products
    assert units["stages"] + units["error"] == 290


def test_oracle_matrix_form_overcounts(counter):
    """The oracle's own arithmetic per evaluation on a few pixels of the 1024^2 Kerr a = 0.9 image:
    several times the Carter-form figure (it builds the full inverse metric
    and its derivatives, multiplies zero tableau entries and recomputes the
    metric for H), so it is reported, not used."""
    import bench
    pix = [100 * 1024 + 300, 512 * 1024 + 512, 700 * 1024 + 900]
    out = subprocess.run([counter, "oracle", "1024", "1024", "12", "0.9", repr(math.radians(60.0)), "1000", "1"]
                         + [str(p) for p in pix], capture_output=True, text=True, check=True).stdout
    d = json.loads(out)
    o = O.trace_pixels(O.Setup(**dict(__import__("paper_2202_00086_amd.workloads", fromlist=["W"]).kerr_ring(0.9))),
                       np.array(pix, np.int32))
    assert d["evals"] == int(o["n_evals"].sum()) and d["steps"] == int(o["n_steps"].sum())
    per_eval = d["flop"] / d["evals"]
    carter = bench.flop_per_launch(d["evals"], d["evals"] - len(pix), d["steps"], src_on=True) / d["evals"]
    assert 100.0 < carter < 125.0
    assert per_eval > 3.0 * carter
