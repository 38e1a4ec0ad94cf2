"""Host arithmetic of the finite-size study (paper_1810_06800_amd.finite_size):
means, straight-line fits and the extrapolations of Eqs. 9-10, on synthetic
numbers with known answers, and the table assembly on a stand-in engine."""
import math

import pytest

from paper_1810_06800_amd import finite_size as fs


def test_mean_sem():
    m, e = fs.mean_sem([1.0, 2.0, 3.0, 4.0])
    assert m == 2.5 and e == pytest.approx(math.sqrt(5 / 3 / 4))


def test_line_fit_exact():
    xs = [0.1, 0.2, 0.5, 0.9]
    a, b, _ = fs.line_fit(xs, [0.3 - 2 * x for x in xs])
    assert a == pytest.approx(0.3) and b == pytest.approx(-2.0)


def test_extrapolations_recover_the_limit():
    # p_c(L) = 0.5 - 0.3 (L/k)^(-3/4)  (Eq. 9, nu = 4/3);  p_j(L) = 0.75 + 2/L  (Eq. 10)
    k = 8
    pts_c = [(r * k, k, 0.5 - 0.3 * r ** -0.75, 0.001) for r in (16, 32, 64)]
    pts_j = [(r * k, k, 0.75 + 2.0 / (r * k), 0.001) for r in (16, 32, 64)]
    assert fs.extrapolate(pts_c, "pc")["value"] == pytest.approx(0.5, abs=1e-12)
    assert fs.extrapolate(pts_j, "pj")["value"] == pytest.approx(0.75, abs=1e-12)
    # no spread at all (k = 1 jams every site): the exact cells pin the fit
    f = fs.extrapolate([(32, 1, 1.0, 0.0), (64, 1, 1.0, 0.0)], "pj")
    assert f["value"] == pytest.approx(1.0) and f["stderr"] < 1e-5


def test_run_grid_on_a_stand_in():
    class Stand:
        def run(self, descs):
            # every run: n_any = L^2/(2k), n_jam = 3 L^2/(4k)
            return [{"status": 0, "n_wrap_any": d[0] * d[0] // (2 * d[1]),
                     "n_jam": 3 * d[0] * d[0] // (4 * d[1])} for d in descs]

    rows = fs.run_grid(Stand(), [2, 4], [16, 32], samples=5)
    assert [(r["k"], r["L"]) for r in rows] == [(2, 32), (2, 64), (4, 64), (4, 128)]
    assert all(r["pc"] == pytest.approx(0.5) and r["pj"] == pytest.approx(0.75) for r in rows)
    f = fs.fits(rows)
    assert f[2]["pc_inf"]["value"] == pytest.approx(0.5) and f[4]["pj_inf"]["value"] == pytest.approx(0.75)
