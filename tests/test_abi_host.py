"""Host-side checks of the C ABI (no GPU needed).

* the built library exports every function include/bls.h declares;
* the ctypes structures match the C layout (sizes and offsets, via gcc);
* the width rule of the library agrees with the oracle's on many inputs;
* status strings, and plan creation failing cleanly without a device.
"""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bls.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1112_1701_amd import _lib
    return _lib.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bls_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert "bls_search" in names and "bls_plan_create" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_c():
    from paper_1112_1701_amd import _lib as L
    structs = {"bls_plan_config": L.BlsPlanConfig, "bls_batch": L.BlsBatch,
               "bls_results": L.BlsResults,
               "bls_device_results": L.BlsDeviceResults,
               "bls_call_stats": L.BlsCallStats,
               "bls_detection": L.BlsDetection,
               "bls_variability_config": L.BlsVariabilityConfig,
               "bls_variability_results": L.BlsVariabilityResults,
               "bls_unbinned_results": L.BlsUnbinnedResults,
               "bls_recovery_config": L.BlsRecoveryConfig,
               "bls_recovery_results": L.BlsRecoveryResults}
    text = open(HEADER).read()
    for opt, cls in (("bls_request", L.BlsRequest),
                     ("bls_result", L.BlsResult),
                     ("bls_server_stats", L.BlsServerStats),
                     ("bls_server_config", L.BlsServerConfig)):
        if re.search(r"}\s*%s\s*;" % opt, text):
            structs[opt] = cls
    lines = ['#include <stdio.h>', '#include <stddef.h>',
             '#include "bls.h"', 'int main(void) {']
    for cname, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));'
                         % (cname, f, cname, f))
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"),
                               src, "-o", exe])
        out = subprocess.check_output([exe]).decode().split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    for cname, cls in structs.items():
        assert int(got[cname + " size"]) == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(cls, f).offset, \
                (cname, f)


@pytest.mark.parametrize("seed", range(3))
def test_width_rule_matches_oracle(lib, seed):
    import paper_1112_1701_amd as bls
    rng = np.random.default_rng(seed)
    t = np.linspace(0, 10, 20)
    x = np.sin(t)
    for _ in range(60):
        nbins = int(rng.integers(2, 5000))
        qmin = float(rng.choice([rng.uniform(1e-4, 0.2), 0.01, 0.005,
                                 1.0 / nbins, 0.5 / nbins]))
        qmax = float(min(0.999, qmin + rng.uniform(0, 0.5)))
        try:
            r = oracle.search(t, x, None, [1.0], nbins, qmin, qmax)
            expect = (r.kmin, r.kmax)
        except oracle.OracleError:
            expect = None
        try:
            got = bls.bls_width_range(nbins, qmin, qmax)
        except bls.BlsError:
            got = None
        assert got == expect, (nbins, qmin, qmax)


def test_status_strings(lib):
    import paper_1112_1701_amd as bls
    assert bls.bls_status_string(0) == "ok"
    for s in range(-6, 0):
        assert bls.bls_status_string(s) not in ("ok", "unknown status")
    assert bls.bls_status_string(-99) == "unknown status"


def test_noalloc_without_device_fails_cleanly(lib):
    """The plan-free search checks its arguments on the host, then needs a
    current device; without one it fails with a status, not a crash."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1112_1701_amd as bls
    from paper_1112_1701_amd import _lib as L
    b = L.BlsBatch()
    o = L.BlsDeviceResults()
    assert lib.bls_search_device_noalloc(None, None, 0, 1, None) == \
        bls.BLS_ERR_INVALID_ARG
    o.sr = o.depth = o.jstart = o.kwidth = o.best_index = 8
    assert lib.bls_search_device_noalloc(C.byref(b), C.byref(o), 1 << 5, 1,
                                         None) == bls.BLS_ERR_INVALID_ARG
    assert "flags" in bls.bls_last_error(None)
    assert lib.bls_search_device_noalloc(C.byref(b), C.byref(o), 0, 1,
                                         None) == bls.BLS_ERR_DEVICE


def test_plan_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1112_1701_amd as bls
    with pytest.raises(bls.BlsError) as ei:
        bls.bls_plan_create()
    assert ei.value.status == bls.BLS_ERR_DEVICE
    assert "device" in bls.bls_last_error(None)


def test_bad_plan_config_rejected_before_device(lib):
    import paper_1112_1701_amd as bls
    with pytest.raises(bls.BlsError) as ei:
        bls.bls_plan_create(max_nbins=5000)
    assert ei.value.status == bls.BLS_ERR_INVALID_ARG
