"""The cost model against the worked arithmetic printed in the paper (tests/golden)."""
import json
import os

import pytest

from paper_1210_7683_amd import costmodel as cm

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_cost_arithmetic.json")))


def close(a, b, tol):
    return abs(a - b) <= tol * abs(b)


def test_per_gls_flops():
    g = G["per_gls_flops"]
    assert cm.flops_per_gls_paper(g["n"], g["p"]) == g["value"]


def test_total_flops_and_hours():
    g = G["total_flops"]
    tot = cm.grid_flops_paper(g["n"], g["p"], g["m"], g["t"])
    assert close(tot, g["value"], g["rel_tol"])
    h = G["hours_at_25_gflops"]
    assert close(tot / (h["gflops"] * 1e9) / 3600, h["value_hours"], h["rel_tol"])


def test_naive_traffic_and_time():
    g, h = G["naive_traffic"], G["naive_io_hours"]
    by = cm.naive_stream_bytes(1000, 10**6, 10**5)
    assert close(by, g["value_bytes"], g["rel_tol"])
    assert close(by / h["bw"] / 3600, h["value_hours"], 0.01)


def test_output_volume():
    g = G["output_written"]
    assert close(cm.output_bytes(10**6, 10**5, 4, 8), g["value_bytes"], g["rel_tol"])


def test_eq_nb():
    g = G["eq_nb"]
    lhs = g["n"] / g["gemm_flops"] * 1e9
    rhs = g["itemsize"] / g["bw"] * 1e9
    assert round(lhs, 2) == g["lhs_ns"] and rhs == g["rhs_ns"]
    assert cm.eq_nb_holds(g["n"], g["gemm_flops"], g["itemsize"], g["bw"])
    assert not cm.eq_nb_holds(g["n"], 260e9, g["itemsize"], g["bw"])


def test_eq_tb():
    g = G["eq_tb"]
    tb = cm.min_tb_exact(g["n"], g["p"], g["tile_flops"], g["itemsize"], g["bw"])
    # the paper rounds the bound 9.43 up to "tb > 10"
    assert tb == g["tb_bound"]
    assert not cm.eq_tb_holds(tb - 1, g["n"], g["p"], g["tile_flops"], g["itemsize"], g["bw"])
    assert cm.eq_tb_holds(tb, g["n"], g["p"], g["tile_flops"], g["itemsize"], g["bw"])


def test_contraction_count_and_ratio_shape():
    assert cm.flops_per_gls_contraction(1000, 4) == 10_000
    assert cm.rotation_flops(1000, 10**6) == 2 * 10**12
    assert cm.tile_ratio(1, 1000, 4) == pytest.approx(4000 / 1004)
    assert cm.tile_ratio(10**6, 1000, 4) == pytest.approx(1000, rel=1e-3)
