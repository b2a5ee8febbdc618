"""CPU-only checks of the C-ABI library: it loads, exports every declared entry
point, and its host-side parameter logic agrees with the oracle's (no GPU call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT, params

HEADER = os.path.join(ROOT, "include", "gvom.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*((?:map|sgt)_[a-z_0-9]+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2109_13176_amd import gvom
    if not os.path.exists(gvom.LIB_PATH):
        from paper_2109_13176_amd import build
        build.build()
    return gvom


def test_header_symbols_exported(lib):
    names = declared_functions()
    assert len(names) >= 14, names
    L = ctypes.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lib.EXPORTED)


def test_status_strings(lib):
    for s in range(0, -8, -1):
        assert lib.map_status_str(s) != "unknown status"
    assert lib.map_status_str(-99) == "unknown status"


def test_params_validate_matches_oracle(lib, orc):
    rng = np.random.default_rng(0)
    cases = [params(512, 512, 64, 0.2), params(1024, 1024, 96, 0.1), params(128, 128, 32, 0.4),
             params(256, 256, 48, 0.4)]
    for _ in range(300):
        p = params(int(rng.integers(1, 40)) * 2, int(rng.integers(1, 40)) * 2,
                   int(rng.integers(0, 140)), float(rng.choice([0.05, 0.1, 0.2, 0.3, 0.4, 0.45])),
                   szv=int(rng.integers(-1, 40)),
                   obs_min_m=float(rng.uniform(0, 1)), obs_max_m=float(rng.uniform(0, 3)),
                   dens_num=int(rng.integers(-1, 4)), dens_den=int(rng.integers(-1, 4)),
                   fit_n=int(rng.integers(0, 17)), neg_thresh_m=float(rng.uniform(-0.1, 1)),
                   neg_search_m=float(rng.uniform(0, 30)))
        cases.append(p)
    for p in cases:
        sg, dg = lib.map_params_validate(p)
        so, do = orc.derive(p)
        assert sg == so, p
        if sg == 0:
            for k in ("n_lo", "n_hi", "tau_neg_q", "search_d", "half_fit"):
                assert dg[k] == do[k], (k, p)
            assert np.float32(dg["inv_r"]) == np.float32(do["inv_r"])


def test_no_cpu_fallback(lib):
    """The binding refuses host tensors: there is no CPU path."""
    import torch
    with pytest.raises((TypeError, RuntimeError)):
        lib.map_insert_scan(ctypes.c_void_p(1), torch.zeros((4, 3)), np.eye(3, 4), 0)
