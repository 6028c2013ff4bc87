"""The byte/flop accounting reproduces the performance numbers the paper prints."""
import json
import os

import pytest

from paper_1103_1363_amd import roofline

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_model.json")))


def test_su3vecmul_example():
    g = GOLD["su3vecmul"]
    # 18 complex loaded + 9 stored, double precision (16 B per complex)
    nbytes = (18 + 9) * 16
    assert nbytes == g["bytes_per_element"]
    assert round(nbytes / g["mem_bandwidth_GBs"]) == g["ns_per_element_memory"]
    assert round(g["fma_per_element"] / g["clock_GHz"] / g["cores"], 1) == g["ns_per_element_fp"]


@pytest.mark.parametrize("prec,peak", [("f32", "peak_sp_GFs"), ("f64", "peak_dp_GFs")])
def test_wilson_bound_is_34_percent(prec, peak):
    """Full-lattice Wilson mat-vec with perfect reuse: 1320 flops per site
    against four 18-real links plus one spinor in and one out."""
    g = GOLD["wilson_bound"]
    eps = roofline.fp_efficiency(roofline.DSLASH_FLOPS,
                                 roofline.full_lattice_dslash_bytes(prec, 18),
                                 g["mem_bandwidth_GBs"] * 1e9, g[peak] * 1e9)
    assert round(100 * eps) == g["eps_fp_percent"]


@pytest.mark.parametrize("row", range(3))
def test_sap_model_reproduces_table(row):
    g = GOLD["sap_table"]
    r = g["rows"][row]
    e = roofline.sap_efficiency(r["eps_bs"], r["t_fp"], r["t_lm"], r["t_tnw_15"], g["eps_lm"])
    # the printed eps_bs is rounded to a whole percent: allow that rounding
    lo = roofline.sap_efficiency(r["eps_bs"] - 0.005, r["t_fp"], r["t_lm"], r["t_tnw_15"], g["eps_lm"])
    hi = roofline.sap_efficiency(r["eps_bs"] + 0.005, r["t_fp"], r["t_lm"], r["t_tnw_15"], g["eps_lm"])
    assert lo - 0.0005 <= r["eps_msap_e"] <= hi + 0.0005
    assert abs(e - r["eps_msap_e"]) < 0.005


def test_compulsory_bytes_per_site():
    assert roofline.dslash_bytes("f64") == 1152
    assert roofline.dslash_bytes("f32") == 576
    assert roofline.dslash_bytes("f16") == 296
    assert roofline.dslash_bytes("f16", nrhs=12) == 1440
    assert roofline.DSLASH_FLOPS == 1320
    assert roofline.CLOVER_FLOPS == 504
