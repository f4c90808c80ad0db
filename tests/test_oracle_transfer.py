"""Pins for the oracle's lattice transfers (Section "Multigrid Solution").

For odd sides (2m+1) the coarse P1 space is nested in the fine one, so the
prolongation must be exact on coarse linear functions, and the Galerkin
products P^T A_f P and (P^T M_f P) 1 must reproduce the coarse stiffness and
lumped mass assembled directly at spacing 2h.  Restriction is checked to be
the exact transpose, and prolongation a partition of unity for any side.
"""
import numpy as np
import pytest

from test_oracle_assembly import dense_A


def P_matrix(orc, Wf, Hf):
    Wc, Hc = (Wf + 1) // 2, (Hf + 1) // 2
    cols = []
    for k in range(Wc * Hc):
        e = np.zeros((1, Hc, Wc))
        e.flat[k] = 1.0
        cols.append(orc.prolong(e, Wf, Hf).ravel())
    return np.stack(cols, 1)


@pytest.mark.parametrize("Wf,Hf", [(9, 7), (17, 5), (8, 6), (10, 11), (2, 3)])
def test_partition_of_unity_and_transpose(orc, Wf, Hf):
    P = P_matrix(orc, Wf, Hf)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-15)
    rng = np.random.default_rng(0)
    vf = rng.normal(size=(3, Hf, Wf))
    vc = orc.restrict(vf)
    for i in range(3):
        assert np.allclose(vc[i].ravel(), P.T @ vf[i].ravel(), atol=1e-13)


@pytest.mark.parametrize("Wf,Hf", [(9, 7), (17, 5), (5, 5)])
def test_nested_odd_sides(orc, Wf, Hf):
    Wc, Hc = (Wf + 1) // 2, (Hf + 1) // 2
    # exact on coarse linear functions
    Xc, Yc = np.meshgrid(np.arange(Wc) * 2.0, np.arange(Hc) * 2.0)
    Xf, Yf = np.meshgrid(np.arange(Wf) * 1.0, np.arange(Hf) * 1.0)
    vc = (0.3 + 1.5 * Xc - 0.7 * Yc)[None]
    vf = orc.prolong(vc, Wf, Hf)[0]
    assert np.allclose(vf, 0.3 + 1.5 * Xf - 0.7 * Yf, atol=1e-13)
    # Galerkin: P^T A_f P = A_c, row-lumped P^T M_f P = M_c (coarse spacing 2h)
    h = 0.1
    P = P_matrix(orc, Wf, Hf)
    mf, sf = orc.assemble(Wf, Hf, h)
    mc, sc = orc.assemble(Wc, Hc, 2 * h)
    assert np.allclose(P.T @ dense_A(sf) @ P, dense_A(sc), atol=1e-12)
    assert np.allclose(P.T @ np.diag(mf.ravel()) @ P @ np.ones(Wc * Hc), mc.ravel(), atol=1e-14)


def test_even_side_edge_rule(orc):
    # the fine node past the last coarse node copies that node (constant extension)
    Wf, Hf = 8, 8
    vc = np.random.default_rng(1).normal(size=(1, 4, 4))
    vf = orc.prolong(vc, Wf, Hf)[0]
    assert np.allclose(vf[::2, ::2], vc[0])
    assert np.allclose(vf[0:7:2, 7], vc[0, :, 3])
    assert np.allclose(vf[7, 0:7:2], vc[0, 3, :])
    assert vf[7, 7] == pytest.approx(vc[0, 3, 3])
