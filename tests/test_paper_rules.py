"""Parameter rules and instance shapes pinned to values the paper prints."""
import json
import math
import os

import numpy as np
import pytest

import sdpgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_rank_rule_table2():
    """Section 5.1's initial rank 2 log m is round(2 ln m) for every row of
    Table 2 (ceil, floor or log2 each miss at least one row)."""
    for name, n, m, r_log, r_sqrt in _load("table2_ranks.json")["rows"]:
        assert sdpgen.rank_rule_2lnm(m) == r_log, name
        assert sdpgen.rank_rule_sqrt2m(m) == r_sqrt, name
    rows = _load("table2_ranks.json")["rows"]
    assert any(math.ceil(2 * math.log(m)) != r for _, _, m, r, _ in rows)
    assert any(math.floor(2 * math.log(m)) != r for _, _, m, r, _ in rows)


def test_table3_nr_column():
    for name, n, m, nr in _load("table3_nr.json")["rows"]:
        assert round(n * math.sqrt(2 * m)) == nr, name


def test_mc_generator_matches_table5():
    """800 (n/2) uniform draws with replacement from an (n/2) x (n/2) grid,
    deduplicated, reproduce every m of Table 5 within 3 standard deviations."""
    for n, m in _load("table5_mc.json")["rows"]:
        d = n // 2
        k = 800 * d
        cells = d * d
        e = sdpgen.mc_sample_count(d, k)
        p = 1 - math.exp(k * math.log1p(-1 / cells))
        sd = math.sqrt(cells * p * (1 - p))
        assert abs(m - e) <= 3 * sd, (n, m, e)


def test_mc_sampler_realisation():
    p = sdpgen.mc_paper_sample(2000, 7)
    d = 1000
    e = sdpgen.mc_sample_count(d, 800 * d)
    assert abs(p.m - e) <= 4 * math.sqrt(e * 0.5)
    assert p.m == np.unique(p.a_row.astype(np.int64) * p.n + p.a_col).size


def test_generators_shapes():
    p = sdpgen.maxcut_torus(10, 10, 1, "unit")
    assert len(p.meta["edges"][0]) == 200
    deg = np.bincount(np.concatenate(p.meta["edges"][:2]), minlength=100)
    assert np.all(deg == 4)
    q = sdpgen.maxcut_gnm(500, 1500, 2)
    assert len(q.meta["edges"][0]) == 1500
    mc = sdpgen.mc_planted(100, 80, 5, 3, count=1234)
    assert mc.m == 1234 and mc.n == 180
    again = sdpgen.mc_planted(100, 80, 5, 3, count=1234)
    assert np.array_equal(mc.a_row, again.a_row) and np.array_equal(mc.b, again.b)
