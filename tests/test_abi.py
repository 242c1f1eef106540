"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/gridplan.h, and rejects bad arguments on the host before
any device call."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2410_13055_amd import cases
from paper_2410_13055_amd import gridplan as gpb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gridplan.h")


def _lib():
    try:
        return gpb.load()
    except gpb.NotBuiltError:
        pytest.skip("libgridplan.so not built")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("plan_init", "dispatch_solve_batch", "dispatch_grad", "plan_step"):
        assert n in names
    assert set(names) == set(gpb.EXPORTS)


def test_library_exports_every_declared_symbol():
    _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", gpb.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in declared_functions():
        assert n in syms, n


def _init(case, opts=None):
    lib = _lib()
    d = gpb._Descriptor(case)
    h = C.c_void_p()
    rc = lib.plan_init(C.byref(h), C.byref(d.desc), C.byref(opts or gpb.options()), None)
    return rc, lib.plan_last_error(None).decode(), d


@pytest.mark.parametrize("mutate,needle", [
    (lambda c: setattr(c.networks[0], "line_to", c.networks[0].line_from.copy()), "endpoints"),
    (lambda c: c.networks[0].gen_node.__setitem__(0, 99), "bad node"),
    (lambda c: c.networks[0].line_beta.__setitem__(0, -1.0), "susceptance"),
    (lambda c: c.networks[0].gen_cost.__setitem__(1, np.nan), "cost"),
    (lambda c: c.networks[0].eta_max.__setitem__(0, -5.0), "box"),
    (lambda c: c.scenarios[0].avail.__setitem__((0, 0), 1.5), "availability"),
    (lambda c: c.scenarios[0].load.__setitem__((0, 0), np.inf), "load"),
    (lambda c: setattr(c, "r", 0.0), "regulariser"),
    (lambda c: setattr(c, "eff", 1.5), "eff"),
    (lambda c: setattr(c.scenarios[0], "network", 3), "network"),
    (lambda c: c.networks[0].eta_min.__setitem__(-1, 0.0), "battery 1: capacity lower bound"),
    (lambda c: setattr(c.networks[0], "n_hvdc", c.networks[0].n_lines + 1), "bad counts"),
    (lambda c: setattr(c.networks[0], "n_hvdc", -1), "bad counts"),
    (lambda c: setattr(c.networks[0], "beta_scales", 2), "beta_scales"),
    (lambda c: (setattr(c.networks[0], "beta_scales", True), c.networks[0].eta_min.__setitem__(12, 0.0)),
     "scaling susceptance needs eta_min > 0"),
])
def test_plan_init_rejects_bad_case(mutate, needle):
    cs = cases.config0()
    mutate(cs)
    rc, msg, _ = _init(cs)
    assert rc == gpb.GP_EINVAL
    assert needle in msg


def test_hvdc_link_susceptance_is_not_read():
    # an HVDC link has no power-flow row: a zero or negative beta on it must
    # not fail validation (on a host without a GPU the call then fails at
    # the first device allocation instead)
    cs = cases.hvdc_two_node()
    cs.networks[0].line_beta[:] = 0.0
    rc, msg, _ = _init(cs)
    assert "susceptance" not in msg
    cs = cases.two_node()
    cs.networks[0].line_beta[:] = 0.0
    rc, msg, _ = _init(cs)
    assert rc == gpb.GP_EINVAL and "susceptance" in msg


@pytest.mark.parametrize("opts,needle", [
    (dict(block=100), "block"),
    (dict(variant=3), "variant"),
    (dict(tol=-1.0), "negative"),
    (dict(stall_pct=-5), "negative"),
    (dict(accept_warm=2), "accept_warm"),
    (dict(rho0=float("inf")), "finite"),
])
def test_plan_init_rejects_bad_options(opts, needle):
    rc, msg, _ = _init(cases.config0(), gpb.options(**opts))
    assert rc == gpb.GP_EINVAL and needle in msg


def test_null_arguments():
    lib = _lib()
    assert lib.plan_init(None, None, None, None) == gpb.GP_EINVAL
    h = C.c_void_p()
    assert lib.plan_init(C.byref(h), None, None, None) == gpb.GP_EINVAL
    assert b"NULL" in lib.plan_last_error(None)
    assert lib.dispatch_solve_batch(None, None, None, 0, 0, None, None) == gpb.GP_EINVAL
    assert lib.dispatch_grad(None, None, None, 0, 0.0, None, None) == gpb.GP_EINVAL
    assert lib.dispatch_objective(None, None, None, 0, 0.0, None) == gpb.GP_EINVAL
    assert lib.plan_set_price_weight(None, 1.0) == gpb.GP_EINVAL
    lib.plan_free(None)


def test_oracle_not_imported_by_product():
    """The product path never imports the oracle."""
    import ast
    pkg = os.path.join(ROOT, "paper_2410_13055_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(dp, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        assert not any(a.name.split(".")[0] == "oracle" for a in node.names), f
                    if isinstance(node, ast.ImportFrom):
                        assert (node.module or "").split(".")[0] != "oracle", f
