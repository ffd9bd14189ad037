"""The C-ABI library loads and exports every entry point include/jet.h declares; host-side argument
checks answer without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "jet.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(jet_[a-z0-9_]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("jet_init", "jet_refine", "jet_rebalance", "jet_km1", "jet_free"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2504_12013_amd import jet
    L = jet.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(jet.EXPORTED) == set(declared_functions())


def test_option_constants_match_header():
    """Every JET_OPT_* the header defines has the same value in the Python binding."""
    from paper_2504_12013_amd import jet
    txt = open(os.path.join(ROOT, "include", "jet.h")).read()
    opts = dict((k, int(v)) for k, v in re.findall(r"^#define\s+(JET_OPT_[A-Z0-9_]+)\s+(\d+)", txt, flags=re.M))
    assert "JET_OPT_SEL_SPLIT_MIN" in opts and len(opts) >= 5
    for name, value in opts.items():
        assert getattr(jet, name) == value, name


def test_defaults_and_error_strings():
    from paper_2504_12013_amd import jet
    p = jet.jet_params_default()
    assert (p.limit, p.max_iters, p.num_tau, p.deadzone_ppm, p.max_rebalance_rounds) == (8, 1000, 3, 100000, 64)
    assert list(p.tau)[:3] == [0.75, 0.375, 0.0]
    L = jet.lib()
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert L.jet_strerror(code)


@pytest.mark.parametrize("n,m,p,k,eps", [(0, 1, 1, 2, 0.03), (1, 0, 1, 2, 0.03), (4, 2, 0, 2, 0.03),
                                          (4, 2, 4, 1, 0.03), (4, 2, 4, 129, 0.03), (4, 2, 4, 2, 0.0),
                                          (4, 2, 4, 2, 1.0)])
def test_init_rejects_bad_scalars_without_gpu(n, m, p, k, eps):
    from paper_2504_12013_amd import jet
    L = jet.lib()
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)   # never dereferenced: scalar checks come first
    rc = L.jet_init(ctypes.byref(h), n, m, p, dummy, dummy, None, None, k, eps, None)
    assert rc == jet.JET_EINVAL
    assert h.value is None
    assert L.jet_last_error(None)


def test_init_rejects_too_many_pins_and_null_arrays():
    from paper_2504_12013_amd import jet
    L = jet.lib()
    h = ctypes.c_void_p()
    assert L.jet_init(ctypes.byref(h), 4, 2, 2**31, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None, 2, 0.03,
                      None) == jet.JET_EOVERFLOW
    assert L.jet_init(ctypes.byref(h), 4, 2, 4, None, None, None, None, 2, 0.03, None) == jet.JET_EINVAL


def test_null_context_calls():
    from paper_2504_12013_amd import jet
    L = jet.lib()
    assert L.jet_free(None) == 0
    assert L.jet_refine(None, None, None, None) == jet.JET_EINVAL
    assert L.jet_km1(None, None, None) == jet.JET_EINVAL


def test_tau_features_host_function():
    """jet_tau_features is host arithmetic: check it against the formulas it documents."""
    import math

    from paper_2504_12013_amd import jet
    st = [1000, 2000, 8000, 10, 4, 1000, 258, 260, 300, 400, 2000, 500, 300, 250, 0, 0]
    f = jet.jet_tau_features(st, 0.03, 2, 12, 4000, 1, 3, 0.1)
    expect = [math.log2(1000), math.log2(2000), math.log2(8000), 4.0, math.log2(10), 8.0, 2.0, 0.03, 2 / 11,
              2.0, 260 / 258 - 1, 300 / 2000, 400 / 2000, 0.5, 0.5, 0.1]
    assert np.allclose(f, np.array(expect, dtype=np.float32), rtol=0, atol=0)
    # single level / single round
    f = jet.jet_tau_features(st, 0.03, 0, 1, 1000, 0, 1, 0.0)
    assert f[8] == 0 and f[9] == 0 and f[14] == 0 and f[15] == 0
    for bad in [dict(level=12), dict(rnd=3), dict(n_finest=10)]:
        args = dict(level=2, levels=12, n_finest=4000, rnd=1, rounds=3)
        args.update(bad)
        with pytest.raises(jet.JetError):
            jet.jet_tau_features(st, 0.03, args["level"], args["levels"], args["n_finest"], args["rnd"],
                                 args["rounds"], 0.0)


def test_mlp_null_and_bad_arguments():
    from paper_2504_12013_amd import jet
    L = jet.lib()
    assert L.jet_mlp_free(None) == 0
    assert L.jet_mlp_forward(None, None, 1, None) == jet.JET_EINVAL
    assert L.jet_mlp_create(None, 0, None) == jet.JET_EINVAL
    assert L.jet_refine_learned(None, None, None, None, 0, 1, 1, None, None, None) == jet.JET_EINVAL
