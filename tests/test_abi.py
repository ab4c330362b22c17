"""The C ABI library loads and exports every symbol include/lorads.h declares;
host-side validation errors are reported before any device call (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import sdpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lorads.h")).read()
    return sorted(set(re.findall(r"\b(lorads_[a-z_A-Z0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2403_09133_amd import lorads
    lib = lorads.load()
    names = _declared()
    assert "lorads_setup" in names and "lorads_admm_solve" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(lorads.EXPORTED) == set(names)


def test_version():
    from paper_2403_09133_amd import lorads
    assert lorads.version().startswith("lorads-gfx950")


def test_default_options():
    from paper_2403_09133_amd import default_options
    o = default_options()
    assert o.eps == 1e-6 and o.rho_max == 5000.0 and o.rho_growth == 1.2 and o.rho_every == 5
    assert o.max_admm_iter == 5000 and o.rank_factor == 1.5 and o.lbfgs_mem == 4


@pytest.mark.parametrize("mutation,msg", [
    (lambda p: setattr(p, "a_row", np.where(np.arange(p.a_nnz) == 0, 10 ** 6, p.a_row)), "out of range"),
    (lambda p: setattr(p, "a_val", np.where(np.arange(p.a_nnz) == 1, np.nan, p.a_val)), "non-finite"),
    (lambda p: setattr(p, "b", np.where(np.arange(p.m) == 2, np.inf, p.b)), "non-finite b"),
    (lambda p: setattr(p, "a_con", np.where(np.arange(p.a_nnz) == 0, p.m + 5, p.a_con)), "constraint id"),
    (lambda p: setattr(p, "c_col", np.where(np.arange(p.c_nnz) == 0, -1, p.c_col)), "out of range"),
    (lambda p: setattr(p, "mu", -0.5), "mu must be finite and >= 0"),
    (lambda p: setattr(p, "mu", float("nan")), "mu must be finite and >= 0"),
])
def test_setup_rejects_malformed_input_on_host(mutation, msg):
    from paper_2403_09133_amd import Context, lorads
    p = sdpgen.maxcut_er(20, 0.3, 1)
    mutation(p)
    with pytest.raises(lorads.LoradsError) as e:
        Context(p)
    assert e.value.status == lorads.LORADS_EINVAL
    assert msg in str(e.value)


def test_setup_rejects_below_diagonal():
    from paper_2403_09133_amd import Context, lorads
    p = sdpgen.mc_planted(5, 5, 1, 2, count=10)
    p.a_row, p.a_col = p.a_col.copy(), p.a_row.copy()
    with pytest.raises(lorads.LoradsError) as e:
        Context(p)
    assert e.value.status == lorads.LORADS_EINVAL and "below the diagonal" in str(e.value)


def test_setup_rejects_empty_constraint():
    from paper_2403_09133_amd import Context, lorads
    p = sdpgen.maxcut_er(10, 0.3, 1)
    p.m = 11
    p.b = np.ones(11)
    with pytest.raises(lorads.LoradsError) as e:
        Context(p)
    assert "has no triplet" in str(e.value)
