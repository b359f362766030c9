"""Pins of the oracle's exact F2M optimum (min-cost flow on the double
cover) against independent exact routes: brute force over {0,1/2,1} edge
vectors (half-integrality, Sec. 4), an exact-rational simplex on the F2M LP
as stated in Sec. 4, scipy's HiGHS, and closed forms."""
import numpy as np
import pytest

from oracle import core, exact
from paper_2011_08170_amd import instances as I


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7])
def test_brute_force_matches_mcf_and_simplex(n):
    for seed in range(4):
        xy = I.uniform(n, 200, 100 * n + seed)
        b = exact.brute_force_opt2(xy)
        assert b == core.exact_opt2(xy) == exact.simplex_opt2(xy)


def test_brute_force_with_duplicate_points():
    xy = I.with_duplicates(7, 50, 2, 3)
    assert exact.brute_force_opt2(xy) == core.exact_opt2(xy)


def test_simplex_matches_mcf_n20():
    for seed in (1, 2):
        xy = I.uniform(20, 1000, seed)
        assert exact.simplex_opt2(xy) == core.exact_opt2(xy)


def test_highs_matches_mcf():
    for n, seed in [(60, 1), (150, 2), (300, 3)]:
        xy = I.clustered(n, 100000, seed, centres=5)
        assert exact.highs_opt2(xy) == core.exact_opt2(xy)


@pytest.mark.parametrize("k1,k2,s", [(2, 2, 10), (4, 3, 7), (6, 5, 13), (8, 8, 3)])
def test_lattice_closed_form(k1, k2, s):
    # k1*k2 even: a Hamiltonian cycle of unit steps exists, and every node
    # pays at least s per unit of degree, so opt = n*s
    xy = I.lattice(k1, k2, s)
    assert core.exact_opt2(xy) == 2 * k1 * k2 * s


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_separated_triangles_closed_form(m):
    xy = I.triangles(m)
    assert core.exact_opt2(xy) == 2 * 30 * m


def test_n3_golden(golden):
    g = golden["n3"]
    assert core.exact_opt2(np.array(g["coords"], np.int32)) == g["opt2"]
    assert exact.brute_force_opt2(np.array(g["coords"], np.int32)) == g["opt2"]


def test_mcf_x_and_lam_certify():
    # the flow's x and potentials form a primal-dual pair: certify must accept
    for n, seed in [(8, 1), (40, 2), (120, 3)]:
        xy = I.uniform(n, 5000, seed)
        opt2, x2, lam = core.exact_opt2(xy, want_x=True)
        eu, ev, ex2 = core.dense_to_edges(x2)
        c = core.certify(xy, lam, eu, ev, ex2)
        assert c["certified"] and c["primal2"] == c["dual2"] == opt2
        assert set(np.unique(ex2)) <= {1, 2}
