"""The paper's test suite as printed (Section 4: the equations of f1..f8 in
Section 4.1 and the run settings of the section's opening paragraph), kept
as a text fixture in tests/golden/paper_suite.txt. The suite builder
(workloads.paper_suite, paper_tolerances) and the oracle's integrand
families are checked against it: each integrand's value at seeded points
of (0,1)^d is computed here from the fixture's constants by the formula the
paper prints, so a wrong constant or cut-off anywhere in the chain (say
f2's 1/50^2, f4's 625 or f6's (3 + i)/10) fails."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_suite.txt")

FAMILY = {"cos_ix": "oscillatory", "prod_peak": "product_peak",
          "corner_ix": "corner_peak", "gauss": "gaussian", "c0": "c0",
          "disc": "discontinuous", "box": "box"}


def _load():
    rows, settings = [], {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            if line[0] == "integrand":
                _, name, dim, form, consts = line[:5]
                kv = {}
                if consts != "-":
                    for item in [consts] + line[5:]:
                        k, v = item.split("=")
                        kv[k] = float(Fraction(v))
                rows.append((name, int(dim), form, kv))
            elif line[0] == "setting":
                settings[line[1]] = float(line[2])
    return rows, settings


ROWS, SETTINGS = _load()


def _printed(form, c, x):
    """The paper's formula for one point x (numpy, float64)."""
    d = len(x)
    i = np.arange(1, d + 1, dtype=np.float64)
    if form == "cos_ix":
        return np.cos(i @ x)
    if form == "prod_peak":
        return np.prod(1.0 / (c["c"] + (x - c["u"]) ** 2))
    if form == "corner_ix":
        return (1.0 + i @ x) ** (-d - 1.0)
    if form == "gauss":
        return np.exp(-c["c"] * np.sum((x - c["u"]) ** 2))
    if form == "c0":
        return np.exp(-c["c"] * np.sum(np.abs(x - c["u"])))
    if form == "disc":
        if np.all(x < (c["o"] + i) / 10.0):
            return np.exp((i + c["s"]) @ x)
        return 0.0
    if form == "box":
        return np.sum(x * x) ** c["p"]
    raise ValueError(form)


def test_fixture_lists_the_suite():
    assert len(ROWS) == 10
    assert sorted({r[0] for r in ROWS}) == [f"f{k}" for k in range(1, 9)]


@pytest.mark.parametrize("name,dim,form,consts", ROWS,
                         ids=[f"{r[0]}_d{r[1]}" for r in ROWS])
def test_suite_integrand_matches_the_printed_one(name, dim, form, consts):
    suite = dict(W.paper_suite())
    wl = suite[f"{name}_d{dim}"]
    assert wl.family == FAMILY[form]
    assert wl.d == dim
    assert np.array_equal(wl.lo, np.zeros(dim)) and np.array_equal(wl.hi, np.ones(dim))
    assert wl.abs_tol == SETTINGS["tau_abs"]
    rng = np.random.default_rng(1000 + 10 * int(name[1:]) + dim)
    pts = list(rng.uniform(0.0, 1.0, size=(24, dim)))
    if form == "disc":
        # points just inside and just outside the cut-off on each axis
        i = np.arange(1, dim + 1)
        cut = (consts["o"] + i) / 10.0
        inner = 0.5 * cut
        pts.append(inner.copy())
        for k in range(dim):
            for off in (-1e-3, 1e-3):
                p = inner.copy()
                p[k] = min(cut[k] + off, 0.999)
                pts.append(p)
    nonzero = 0
    for x in pts:
        want = _printed(form, consts, np.asarray(x, dtype=np.float64))
        got = oracle.f(wl.family, wl.params, x)
        nonzero += want != 0.0
        if want == 0.0:
            assert got == 0.0, (x, got)
        else:
            assert got == pytest.approx(want, rel=1e-12, abs=0.0), (x, got, want)
    assert nonzero > 0


def test_tolerance_sweep_spans_the_printed_range():
    taus = W.paper_tolerances()
    assert taus[0] == SETTINGS["tau_rel_first"]
    assert taus[-1] == pytest.approx(SETTINGS["tau_rel_last"], rel=1e-12)
    # equal ratios between consecutive tolerances (the sweep's reading)
    r = np.array(taus[1:]) / np.array(taus[:-1])
    assert np.allclose(r, r[0], rtol=1e-12) and r[0] < 1.0
