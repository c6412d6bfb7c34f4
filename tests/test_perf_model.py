"""Pins of the deployment model (Eqs. 4-10) to the numbers the paper prints."""

import json
import os

import pytest

from paper_1606_04473_amd import perf_model as pm


@pytest.fixture(scope="module")
def table(golden_dir):
    with open(os.path.join(golden_dir, "table2_model_constants.json")) as f:
        return json.load(f)


def _plat(table, net):
    return pm.from_table(table[net], table["computation_time_1pgpu"], table["power_idle_or_receiving_w"],
                         table["power_computing_w"])


def test_fdr_time_optimum_matches_paper(table):
    p, v, t = pm.best_time(_plat(table, "FDR"))
    assert [p, v] == table["reported_time_optimum"]["FDR"]
    assert abs(t - 1.6828) < 1e-3


def test_qdr_optimum_is_a_near_tie_with_the_paper(table):
    plat = _plat(table, "QDR")
    p, v, t = pm.best_time(plat)
    rp, rv = table["reported_time_optimum"]["QDR"]
    t_paper = plat.exec_time(rp, rv)
    # the grid minimum and the paper's choice differ by well under 0.1%
    assert (t_paper - t) / t < 1e-3
    assert abs(t_paper - 2.4803) < 1e-3


def test_transfer_times_close_to_text(table):
    for net in ("QDR", "FDR"):
        t1 = _plat(table, net).t_transfer(1)
        assert abs(t1 - table["reported_single_gpu_transfer_s"][net]) / t1 < 0.03


def test_energy_optimum_one_pgpu(table):
    plat = _plat(table, "FDR")
    p, v, _ = pm.best_energy(plat, max_p=1, max_v_per_p=table["max_vgpus_per_k20"])
    assert [p, v] == table["reported_energy_optimum_one_pgpu"]


def test_model_closed_forms():
    plat = pm.Platform(10.0, 0.1, 0.0, 0.0, 0.0, 2.0)
    assert plat.t_transfer(4) == pytest.approx(2.4)
    assert plat.time_not_overlapped(1, 1) == pytest.approx(12.1)
    assert plat.time_fully_overlapped(1, 2) == pytest.approx(2.2 / 2 + 2 * 5.0)
    assert plat.exec_time(1, 2) == pytest.approx(max(2.2 / 2 + 10.0, 2.2 + 5.0))
    e = plat.energy(2, 1)
    t = plat.exec_time(2, 1)
    assert e == pytest.approx(2 * (5.0 * 102 + (t - 5.0) * 47))
    fit = pm.fit_one_gpu(1.0, 3.0, 0.01)
    assert fit.exec_time(1, 1) == pytest.approx(4.01)
    assert len(pm.tenants_on_one_gpu(fit, 8)) == 8


def test_split_ranges_cover_trials():
    from paper_1606_04473_amd.serving import split_ranges
    for n, v in ((10, 3), (1_000_000, 8), (7, 7), (5, 1)):
        r = split_ranges(n, v)
        assert len(r) == v and r[0][0] == 0
        assert all(b + c == r[i + 1][0] for i, (b, c) in enumerate(r[:-1]))
        assert r[-1][0] + r[-1][1] == n
        assert max(c for _, c in r) - min(c for _, c in r) <= 1


def test_split_model_is_eqs_7_to_10_on_one_gpu():
    from paper_1606_04473_amd.serving import fit_split_model
    m = fit_split_model(transfer_s=0.08, compute_s=0.02, fixed_s=0.001, w_idle=150.0, w_busy=700.0)
    for v in (1, 2, 4, 8):
        tt = v * 0.001 + 0.08                      # Eq. 6: per-tenant costs grow, the split YET does not
        full = tt / v + v * (0.02 / v)             # Eq. 7 with p = 1
        part = tt + 0.02 / v                       # Eq. 8
        assert m.exec_time(1, v) == pytest.approx(max(full, part))   # Eq. 9
        t = max(full, part)
        assert m.energy(1, v) == pytest.approx(0.02 * 700.0 + (t - 0.02) * 150.0)   # Eq. 10
