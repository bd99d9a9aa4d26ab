"""Host logic of the library, without a GPU: the reference data it builds for
every element type and rule (quadrature points and weights, nodal basis
values and gradients at the points) against the oracle's independent
construction.  The library writes the rules in closed form, by Newton's
method or from published digits; the oracle solves their moment equations in
40-digit arithmetic; the bases are evaluated by separate code."""

import numpy as np
import pytest

import oracle
from oracle import quadrature

# (dim, order, points) for every rule each element type accepts
CASES = ([(1, p, q) for p in (1, 2) for q in (2, 3, 5, 6)] + [(1, p, q) for p in (3, 4) for q in (5, 6)] +
         [(2, p, q) for p in (1, 2) for q in (3, 6, 16)] + [(2, p, 16) for p in (3, 4)] +
         [(3, p, q) for p in (1, 2) for q in (4, 11, 35)])


@pytest.fixture(scope="module")
def lf():
    import paper_2605_14035_amd as lf
    return lf


def sort_rule(xi, w):
    order = np.lexsort(np.vstack([np.round(xi.T, 12), np.round(w, 12)]))
    return xi[order], w[order]


@pytest.mark.parametrize("d,p,q", CASES)
def test_rule_and_basis_match_oracle(lf, d, p, q):
    t = lf.lfem_reference_table(d, p, q)
    assert len(t["w"]) == q
    qp, qw = quadrature.rule(d, q)
    a_xi, a_w = sort_rule(t["xi"], t["w"])
    b_xi, b_w = sort_rule(np.asarray(qp, dtype=float).reshape(q, d), np.asarray(qw, dtype=float))
    # the 16-point rule carries the published 15 digits
    tol = 2e-15 if q == 16 else 1e-15
    assert np.abs(a_w - b_w).max() <= tol
    assert np.abs(a_xi - b_xi).max() <= tol
    for i in range(q):
        phi, dphi = oracle.basis(d, p, t["xi"][i])
        assert np.abs(t["phi"][i] - phi).max() <= 1e-13, (i, "phi")
        assert np.abs(t["dphi"][i] - dphi).max() <= 1e-12, (i, "dphi")


def test_defaults(lf):
    want = {(1, 1): 2, (1, 2): 3, (1, 3): 5, (1, 4): 6, (2, 1): 3, (2, 2): 6, (2, 3): 16, (2, 4): 16,
            (3, 1): 4, (3, 2): 11, (3, 3): 35, (3, 4): 35}
    for (d, p), q in want.items():
        assert len(lf.lfem_reference_table(d, p, 0)["w"]) == q


def test_unsupported(lf):
    for d, p, q in ((3, 5, 0), (2, 5, 0), (2, 2, 7), (1, 1, 4)):
        with pytest.raises(lf.LfemError) as e:
            lf.lfem_reference_table(d, p, q)
        assert e.value.status == lf.LFEM_EUNSUPPORTED
