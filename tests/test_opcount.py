"""The host operation count of the cache build's source (physics.h and
solve.h with a counting scalar): it compiles, it counts what the source
does (elastic modes skip the theta_I search, qSH evaluations are cheaper
than the coupled modes', OEV costs more than MEV), and the polish from a
nearby start is accepted."""
import numpy as np

from paper_2609_26108_amd import opcount


def rock_layer1(q=True):
    r = [14.4e6, 4.5e6, 9.0e6, 2.25e6, 3.0e6]
    qs = [30.0, 15.0, 20.0, 15.0, 12.0] if q else [np.inf] * 5
    return np.array(r + qs + [2300.0, 0.0, 0.0])


def test_counts_follow_the_source():
    d = opcount.count(rock_layer1()[None], n_dirs=36, n_sweep=360, mode=1)
    for k in ("MEV", "OEV"):
        assert d[f"{k}_qSH"]["energy_eval_flops"] < d[f"{k}_qP"]["energy_eval_flops"]
        assert d[f"{k}_qP"]["energy_eval_trans"] == 2.0  # sincos and expm1
    assert d["OEV_qP"]["energy_eval_flops"] > d["MEV_qP"]["energy_eval_flops"]
    assert d["MEV_qSV"]["theta_i_solve_flops"] > 5 * d["MEV_qSV"]["energy_eval_flops"]
    b = d["build"]
    assert b["sweep_flops_per_class"] > 360 * d["MEV_qSV"]["energy_eval_flops"]
    assert b["warm_accepted"] > 0.9
    assert 0 < b["warm_flops_per_direction"] < b["solve_flops_per_direction"]


def test_elastic_modes_skip_the_theta_i_search():
    d = opcount.count(rock_layer1(q=False)[None], n_dirs=12, n_sweep=64, mode=0)
    assert d["MEV_qP"]["theta_i_solve_flops"] == 0.0
    assert d["MEV_qP"]["theta_i_found"] == 1.0
