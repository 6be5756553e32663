"""Host logic of the Sec. 5 study driver: case generation, t* and the Fig. 17 slopes."""
import math

import pytest

from paper_2511_10257_amd import studies


def test_sweep_cases_one_field_free_case_per_stefan_number():
    cases = studies.sweep_cases(48, [0.0, 4.0], [0.1, 0.3])
    keys = [(c["case"]["ste"], c["case"]["bo_m"], c["case"]["orientation"]) for c in cases]
    assert keys == [(0.1, 0.0, "none"), (0.1, 4.0, "vertical"), (0.1, 4.0, "horizontal"),
                    (0.3, 0.0, "none"), (0.3, 4.0, "vertical"), (0.3, 4.0, "horizontal")]
    vert = [c for c in cases if c["case"]["orientation"] == "vertical"][0]
    assert vert["angle_deg"] == 90.0 and vert["nx"] == 48 and vert["drop"][2] == 12.0
    air = studies.sweep_cases(48, [0.0], [0.1], gas_lambda_ratio=0.036)[0]
    assert air["lam"][2] == pytest.approx(0.036 * air["lam"][1])
    assert air["lam"][2] / (air["rho"][2] * air["cp"][2]) == pytest.approx(0.4)


def _res(ste, bo, ori, t, fo, hm):
    return dict(case=dict(ste=ste, bo_m=bo, orientation=ori), frozen=True, freeze_t=t, freeze_fo=fo, hm_r0=hm)


def test_t_star_and_scaling_slope():
    res = [_res(0.1, 0.0, "none", 100.0, 1.0, 1.0), _res(0.1, 8.0, "vertical", 110.0, 1.1, 1.05),
           _res(0.1, 8.0, "horizontal", 95.0, 0.95, 0.97), _res(0.3, 8.0, "vertical", 40.0, 0.4, 1.0)]
    ts = {(t["ste"], t["orientation"]): t["t_star"] for t in studies.t_star(res)}
    assert ts == {(0.1, "vertical"): pytest.approx(0.1), (0.1, "horizontal"): pytest.approx(-0.05)}
    # points on H = (Ste Fo)^0.5 give the slope 0.5 exactly
    pts = [_res(s, 0.0, "none", 1.0, fo, math.sqrt(s * fo)) for s, fo in ((0.1, 2.0), (0.2, 3.0), (0.3, 0.7))]
    assert studies.scaling_slope(pts) == pytest.approx(0.5, abs=1e-12)


def test_front_scaling_recovers_a_square_root_rise():
    """Series with Hs/R0 = c sqrt(Ste Fo) (c differing between cases) give the slope 0.5
    per case and pooled; points outside the 10-60% window of the final frozen height and
    cases that did not freeze are left out."""
    import numpy as np
    res = []
    for ste, c in ((0.1, 1.4), (0.2, 1.3), (0.3, 1.5)):
        fo = np.linspace(0.001, 2.0, 400)
        hs = c * np.sqrt(ste * fo)
        hs[-5:] = hs[-6] * np.linspace(2.0, 3.0, 5)      # the apex: the front accelerates
        res.append(dict(case=dict(ste=ste, bo_m=0.0, orientation="none"), frozen=True,
                        series=dict(fo=list(fo), hs_r0=list(hs))))
    res.append(dict(case=dict(ste=0.5, bo_m=0.0, orientation="none"), frozen=False,
                    series=dict(fo=[1.0, 2.0], hs_r0=[5.0, 1.0])))
    out = studies.front_scaling(res)
    assert len(out["cases"]) == 3
    for c in out["cases"]:
        assert c["slope"] == pytest.approx(0.5, abs=1e-9)
    # the prefactors differ between cases, so the pooled slope is 0.5 only approximately
    assert out["slope"] == pytest.approx(0.5, abs=0.05)


def test_write_csv_one_file_per_case(tmp_path):
    res = [dict(case=dict(ste=0.1, bo_m=4.0, orientation="vertical"),
                series=dict(step=[50, 100], fo=[0.01, 0.02], h_r0=[1.0, 1.01], hs_r0=[0.1, 0.15], pe=[2.0, 1.0],
                            q_l=[0.05, 0.1], fl=[0.9, 0.8], wall_heat=[-1.0, -0.9]))]
    (path,) = studies.write_csv(res, str(tmp_path))
    rows = open(path).read().splitlines()
    assert path.endswith("ste0.1_bo4_vertical.csv") and len(rows) == 3
    assert rows[0].startswith("step,fo,ste_fo") and rows[2].split(",")[2] == "0.002"
