"""Pins of the oracle's FP64 discrete adjoint of the heated channel.

The paper has no gradients; the adjoint is pinned by (i) central finite
differences of the oracle's own forward objective at step sizes where the
difference quotient has converged, (ii) the exact Euler identities that follow
from the thermal problem being linear and homogeneous in the wall flux when
the inlet and initial temperatures equal the datum T_ref, and (iii)
independence of the checkpoint interval.
"""
import numpy as np
import pytest

import oracle as O
from paper_2302_04120_amd import workloads as WL

NX, NY, N = 16, 6, 300


def _case():
    prm, ini = WL.adjoint_channel(nx=NX, ny=NY, dx=1e-4, tau_ratio=0.7)
    prm["flux"] = WL.rng(1).uniform(5e3, 1.5e4, NX)
    return prm, ini


def _make(prm, ini):
    ch = O.Chan(NX, NY, prm, bc_x="inlet_outlet", bc_y="walls", thermal=True)
    ch.init(**ini)
    return ch


def _J(prm, ini, wt=1.0, wn=1.0):
    ch = _make(prm, ini)
    ch.step(N)
    return ch.objective(NX // 2, wt, wn)


def test_adjoint_matches_central_differences():
    prm, ini = _case()
    J, gq, gt = _make(prm, ini).adjoint(N, 64, NX // 2)
    assert J == pytest.approx(_J(prm, ini), rel=1e-14)
    for k in (0, 5, 8, 15):
        h = 1e-4 * prm["flux"][k]  # where truncation and FP64 noise are both small
        fp, fm = prm["flux"].copy(), prm["flux"].copy()
        fp[k] += h
        fm[k] -= h
        fd = (_J(dict(prm, flux=fp), ini) - _J(dict(prm, flux=fm), ini)) / (2 * h)
        assert gq[k] == pytest.approx(fd, rel=2e-4, abs=1e-9)
    c = prm["dx"] / prm["dt"]
    cs2 = c * c / 3
    for which, key in ((0, "nu"), (1, "alpha")):
        tau = prm[key] / cs2 + prm["dt"] / 2
        h = 1e-6 * tau
        Jp = _J(dict(prm, **{key: (tau + h - prm["dt"] / 2) * cs2}), ini)
        Jm = _J(dict(prm, **{key: (tau - h - prm["dt"] / 2) * cs2}), ini)
        assert gt[which] == pytest.approx((Jp - Jm) / (2 * h), rel=2e-4)


def test_adjoint_euler_identities():
    """T_out is affine in q'' with T_out(0) = T_in, so sum_k q_k dT_out/dq_k =
    T_out - T_in; Nu is homogeneous of degree 0 in q'', so sum_k q_k dNu/dq_k = 0."""
    prm, ini = _case()
    q = prm["flux"]
    Jt, gt_q, _ = _make(prm, ini).adjoint(N, 50, NX // 2, 1.0, 0.0)
    assert np.dot(q, gt_q) == pytest.approx(Jt - prm["T_in"], rel=1e-9)
    Jn, gn_q, _ = _make(prm, ini).adjoint(N, 50, NX // 2, 0.0, 1.0)
    assert abs(np.dot(q, gn_q)) < 1e-9 * np.abs(q * gn_q).sum()


def test_adjoint_checkpoint_interval_independent():
    prm, ini = _case()
    a = _make(prm, ini).adjoint(N, 7, NX // 2)
    b = _make(prm, ini).adjoint(N, 1000, NX // 2)
    assert a[0] == b[0]
    np.testing.assert_allclose(a[1], b[1], rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(a[2], b[2], rtol=1e-12)
