"""Trend-level checks of the Sec. 5 studies (Figs. 11, 16, 17, 18) on synthetic droplets.

The paper's figures carry no numeric data, so these tests check directions only: the
droplet grows taller while it freezes (the solid is less dense), a vertical field makes
it taller and a horizontal one flatter (Fig. 11), and, with a gas that conducts heat
poorly (air against a water-based ferrofluid: lambda_g / lambda_l ~ 0.036), the
vertical field slows the latent-heat release and the horizontal one speeds it up
(Figs. 16 and 18). Magnitudes are parity-unpinned.
"""
import numpy as np
import pytest

from paper_2511_10257_amd import studies

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sweep():
    cases = studies.sweep_cases(64, [0.0, 16.0], [0.1], gas_lambda_ratio=0.036)
    res = studies.run(cases, chunk=100, max_steps=6800)
    return {(r["case"]["bo_m"], r["case"]["orientation"]): r["series"] for r in res}


def test_droplet_grows_while_freezing(sweep):
    h = np.array(sweep[(0.0, "none")]["h_r0"])
    assert h[-1] > 1.03 and h[-1] > h[len(h) // 4] > h[0] - 1e-3


def test_field_orientation_orders_the_height(sweep):
    v, n, hz = (np.array(sweep[k]["h_r0"]) for k in ((16.0, "vertical"), (0.0, "none"), (16.0, "horizontal")))
    late = slice(5, None)
    assert np.all(v[late] > n[late]) and np.all(n[late] > hz[late])
    assert v[-1] - n[-1] > 0.01 and n[-1] - hz[-1] > 0.01


def test_field_orientation_orders_the_freezing_rate(sweep):
    fl = {k: np.array(sweep[k]["fl"]) for k in sweep}
    ql = {k: np.array(sweep[k]["q_l"]) for k in sweep}
    v, n, hz = (16.0, "vertical"), (0.0, "none"), (16.0, "horizontal")
    # second half of the run: more liquid left under the vertical field, less under the
    # horizontal one; the solid ratio of Eq. 51 the other way round
    half = slice(len(fl[n]) // 2, None)
    assert np.all(fl[v][half] > fl[n][half]) and np.all(fl[n][half] > fl[hz][half])
    assert np.all(ql[v][half] < ql[n][half]) and np.all(ql[n][half] < ql[hz][half])
    for k in sweep:
        assert np.all(np.isfinite(fl[k]))


def test_freezing_front_rises_as_the_square_root_of_ste_fo():
    """Fig. 17 under the front reading: the frozen height along the centre column grows
    as (Ste Fo)^0.5 while the front rises (0.54 here on 64^2, 0.52 on 128^2), with and
    without the field."""
    cases = studies.sweep_cases(64, [0.0, 16.0], [0.1], orientations=("vertical",), gas_lambda_ratio=0.036)
    res = studies.run(cases, chunk=100, max_steps=100000)
    out = studies.front_scaling(res)
    assert len(out["cases"]) == 2
    for c in out["cases"]:
        assert 0.45 < c["slope"] < 0.6, c
        assert c["points"] > 30


def test_deformation_ratio_grows_with_the_magnetic_bond_number():
    """Sec. 4.3 (Fig. 7): a suspended ferrofluid droplet (mu_r 2.2) stretches along a
    vertical field, more for a stronger field; without a field it stays round. The
    experimental ratios are not available, so only the trend is checked."""
    res = {r["bo_m"]: r["b_over_a"] for r in studies.deformation(100, [0.0, 2.0, 4.0], steps=40000, chunk=1000)}
    assert abs(res[0.0] - 1.0) < 1e-3
    assert res[2.0] > 1.05 and res[4.0] > res[2.0] + 0.05
