"""Pins of the oracle's lattice constants and ghost basis against values the
paper prints and against exact identities.  CPU only."""
from fractions import Fraction as Fr
import itertools

import numpy as np
import pytest

from conftest import golden
from oracle import ptrt as O
from oracle import trt_rlb as R

CS2 = 1.0 / 3.0


def test_d2q9_table_matches_printed():
    g = golden("d2q9_lattice.json")
    e, w, opp = O.lattice(O.D2Q9)
    assert list(e[:, 0]) == g["ex"]
    assert list(e[:, 1]) == g["ey"]
    assert (e[:, 2] == 0).all()
    np.testing.assert_allclose(w * 36, g["w_times_36"], rtol=0, atol=1e-14)
    # opposite directions: e_ibar = -e_i, w_ibar = w_i (text after Eq. D2Q9)
    assert (e[opp] == -e).all() and np.allclose(w[opp], w)


def test_d3q19_composition_and_isotropy():
    """App. A.2: 1 rest, 6 axial, 12 face diagonals, no body diagonal.  The
    weights (not printed) are pinned by the moment conditions the Hermite
    equilibrium needs: sum w = 1, sum w e_a e_b = c_s^2 d_ab, fourth-order
    isotropy sum w e_a^2 e_b^2 = c_s^4 (a != b), sum w e_a^4 = 3 c_s^4,
    and odd moments zero."""
    e, w, opp = O.lattice(O.D3Q19)
    n2 = (e ** 2).sum(1)
    assert sorted(np.bincount(n2).tolist()) == sorted([1, 6, 12])
    assert (n2 <= 2).all()
    assert (e[opp] == -e).all() and np.allclose(w[opp], w)
    assert abs(w.sum() - 1) < 1e-15
    for a, b in itertools.product(range(3), repeat=2):
        assert abs((w * e[:, a] * e[:, b]).sum() - CS2 * (a == b)) < 1e-15
        assert abs((w * e[:, a] * e[:, b] ** 2).sum()) < 1e-15
        m4 = (w * e[:, a] ** 2 * e[:, b] ** 2).sum()
        assert abs(m4 - (3 * CS2 ** 2 if a == b else CS2 ** 2)) < 1e-15
    for a, b, c in itertools.product(range(3), repeat=3):
        assert abs((w * e[:, a] * e[:, b] * e[:, c]).sum()) < 1e-15


def test_oracle_and_numpy_tables_agree():
    for lat, name in ((O.D2Q9, "D2Q9"), (O.D3Q19, "D3Q19"), (O.D3Q27, "D3Q27")):
        e, w, _ = O.lattice(lat)
        e2, w2 = R.lattice(name)
        D = e2.shape[1]
        assert (e[:, :D] == e2).all()
        assert np.allclose(w, w2, rtol=0, atol=1e-16)


def test_d2q9_ghost_mode_matches_printed_table():
    """App. A.1: phi values c_s^4 (1, -2 x4, 4 x4) and norm 4 c_s^8; the
    Gram-Schmidt step of the oracle must leave the printed mode unchanged."""
    g = golden("d2q9_lattice.json")
    phi, nrm = O.ghost_basis(O.D2Q9)
    assert phi.shape == (1, 9)
    np.testing.assert_allclose(phi[0], np.array(g["phi_in_units_of_cs4"]) * CS2 ** 2,
                               rtol=0, atol=1e-16)
    assert abs(nrm[0] - g["ghost_norm_in_units_of_cs8"] * CS2 ** 4) < 1e-16


def _symmetric_hydro_modes(e, D):
    rows = [np.ones(len(e))]
    for a in range(D):
        for b in range(a, D):
            rows.append(e[:, a] * e[:, b] - CS2 * (a == b))
    return np.array(rows, dtype=np.float64)


@pytest.mark.parametrize("lat,name", [(O.D2Q9, "D2Q9"), (O.D3Q19, "D3Q19"), (O.D3Q27, "D3Q27")])
def test_subspace_dimensions(lat, name):
    """Tables sym_structure / antisym_structure / lattice_summary."""
    g = golden("subspace_structure.json")[name]
    e, w, opp = O.lattice(lat)
    Q = len(w)
    D = g["D"]
    Q0 = int(((e ** 2).sum(1) == 0).sum())
    Qp = (Q - Q0) // 2
    assert (Q, Q0, Qp) == (g["Q"], g["Q0"], g["Qp"])
    # symmetric / antisymmetric projectors, Eq. parity
    Psym = 0.5 * (np.eye(Q) + np.eye(Q)[opp])
    Panti = 0.5 * (np.eye(Q) - np.eye(Q)[opp])
    assert np.linalg.matrix_rank(Psym) == g["dimS"] == Q0 + Qp
    assert np.linalg.matrix_rank(Panti) == g["dimA"] == Qp
    hyd = _symmetric_hydro_modes(e, D)
    assert np.linalg.matrix_rank(hyd) == g["dimS0"] + g["dimS2"]
    phi, _ = O.ghost_basis(lat)
    assert phi.shape[0] == g["NG"] == g["dimS"] - 1 - D * (D + 1) // 2
    # antisymmetric completeness: H1 and the third-order modes span A
    H1 = e[:, :D].T.astype(float)
    H3 = R.third_order_modes(e[:, :D].astype(float))
    assert np.linalg.matrix_rank(H3) == g["N3"]
    if g["complete"]:
        assert np.linalg.matrix_rank(np.vstack([H1, H3])) == g["dimA"]
    else:
        # D3Q27: the deficit is filled by the fifth-order modes (App. A.3)
        assert np.linalg.matrix_rank(np.vstack([H1, H3])) == g["dimA"] - g["deficit"]
        psi = O.fifth_modes(lat)
        assert np.linalg.matrix_rank(np.vstack([H1, H3, psi])) == g["dimA"]


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19, O.D3Q27])
def test_ghost_basis_orthogonal_and_complete(lat):
    """Eq. S_decomp: the ghost basis is symmetric, orthogonal (weighted) to
    the mass and stress modes and to itself, and with them spans S."""
    e, w, opp = O.lattice(lat)
    D = 2 if lat == O.D2Q9 else 3
    phi, nrm = O.ghost_basis(lat)
    hyd = _symmetric_hydro_modes(e, D)
    for k in range(phi.shape[0]):
        assert np.allclose(phi[k], phi[k][opp], atol=1e-16)  # symmetric
        for h in hyd:
            assert abs((w * phi[k] * h).sum()) < 1e-15
        for m in range(phi.shape[0]):
            ip = (w * phi[k] * phi[m]).sum()
            assert abs(ip - (nrm[k] if k == m else 0.0)) < 1e-15
    Q = len(w)
    Psym = 0.5 * (np.eye(Q) + np.eye(Q)[opp])
    span = np.vstack([hyd, phi])
    assert np.linalg.matrix_rank(span) == np.linalg.matrix_rank(Psym)
    # every symmetric vector lies in the span
    coef, res, *_ = np.linalg.lstsq(span.T, Psym, rcond=None)
    assert np.abs(span.T @ coef - Psym).max() < 1e-12


def test_literal_d3q19_products_are_not_orthogonal():
    """Exact rationals behind reading R3: the three printed D3Q19 products
    overlap each other and the stress modes, so they cannot serve as the
    orthogonal basis of Eq. ghost_proj as printed."""
    e, _, _ = O.lattice(O.D3Q19)
    cs2 = Fr(1, 3)
    w = [Fr(1, 3) if (v ** 2).sum() == 0 else (Fr(1, 18) if (v ** 2).sum() == 1 else Fr(1, 36))
         for v in e]

    def prod(a, b):
        return [(int(v[a]) ** 2 - cs2) * (int(v[b]) ** 2 - cs2) for v in e]

    def dot(p, q):
        return sum(wi * pi * qi for wi, pi, qi in zip(w, p, q))

    pxy, pyz = prod(0, 1), prod(1, 2)
    Hzz = [int(v[2]) ** 2 - cs2 for v in e]
    assert dot(pxy, pxy) == 4 * cs2 ** 4            # the printed norm holds ...
    assert dot(pxy, pyz) == -cs2 ** 4               # ... orthogonality does not
    assert dot(pxy, Hzz) == -cs2 ** 3               # and it overlaps a stress mode


def test_d3q19_third_order_modes_overlap():
    """Exact rationals behind the D3Q19 third-order reading of the NumPy
    TRT-RLB: <H_xxy, H_yzz>_w = -c_s^6 on D3Q19, while the D2Q9 pair
    H_xxy, H_xyy is orthogonal; both have norm 2 c_s^6 (App. A.1, A.2)."""
    cs2 = Fr(1, 3)
    weights = {"D2Q9": (Fr(4, 9), Fr(1, 9), Fr(1, 36)),
               "D3Q19": (Fr(1, 3), Fr(1, 18), Fr(1, 36))}
    for name, expect_cross in (("D2Q9", 0), ("D3Q19", -cs2 ** 3)):
        e, _ = R.lattice(name)
        e = e.astype(int)
        wv = [weights[name][int((v ** 2).sum())] for v in e]
        hxxy = [int(v[1]) * (int(v[0]) ** 2 - cs2) for v in e]
        if name == "D2Q9":
            other = [int(v[0]) * (int(v[1]) ** 2 - cs2) for v in e]  # H_xyy
        else:
            other = [int(v[1]) * (int(v[2]) ** 2 - cs2) for v in e]  # H_yzz
        dot = sum(a * b * c for a, b, c in zip(wv, hxxy, other))
        nrm = sum(a * b * b for a, b in zip(wv, hxxy))
        assert nrm == 2 * cs2 ** 3
        assert dot == expect_cross
