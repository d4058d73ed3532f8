"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/pp.h declares, and rejects bad arguments before touching a device."""
import os
import re

import pytest

from paper_2502_10640_amd import pp
from paper_2502_10640_amd.build import LIB_PATH

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "pp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pp_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB_PATH):
        pytest.fail("libpp_hip.so is not built (run __graft_entry__.build())")
    return pp.load()


def test_every_declared_symbol_is_exported(lib):
    declared = header_functions()
    assert len(declared) >= 15
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    assert set(pp.EXPORTS) == set(declared)


def test_abi_version(lib):
    assert pp.pp_abi_version() == 4


def test_destroy_null_and_last_error(lib):
    assert lib.pp_destroy(None) == pp.PP_OK
    assert isinstance(pp.pp_last_error(None), str)


FAKE = [0x1000 * (k + 1) for k in range(8)]   # never dereferenced: validation fails first


@pytest.mark.parametrize("bunches,n_total,state,prec,msg", [
    ([], 10, FAKE, pp.PP_MIXED, "at least one bunch"),
    ([(0, 10, 1.0, 0.0, 1e-15)], 10, [0] * 8, pp.PP_MIXED, "NULL array"),
    ([(0, 10, 1.0, 0.0, 1e-15)], 10, FAKE, 7, "precision"),
    ([(0, 0, 1.0, 0.0, 1e-15)], 10, FAKE, pp.PP_FP64, "offset/n"),
    ([(5, 10, 1.0, 0.0, 1e-15)], 10, FAKE, pp.PP_FP64, "offset/n"),
    ([(0, 6, 1.0, 0.0, 1e-15), (4, 4, 1.0, 0.0, 1e-15)], 10, FAKE, pp.PP_FP64, "offset/n"),
    ([(0, 10, 0.0, 0.0, 1e-15)], 10, FAKE, pp.PP_MIXED, "weight > 0"),
    ([(0, 10, 1.0, -1.0, 1e-15)], 10, FAKE, pp.PP_MIXED, "softening >= 0"),
    ([(0, 10, 1.0, 0.0, 0.0)], 10, FAKE, pp.PP_MIXED, "dt > 0"),
    ([(0, 10, 1.0, float("nan"), 1e-15)], 10, FAKE, pp.PP_MIXED, "finite"),
    ([(0, 2 ** 30, 1.0, 0.0, 1e-15)], 2 ** 30, FAKE, pp.PP_MIXED, "2^30 or more"),
    ([(0, 10, float("inf"), 0.0, 1e-15)], 10, FAKE, pp.PP_MIXED, "finite"),
    ([(0, 10, 1.0, 0.0, 1e-15)], 0, FAKE, pp.PP_MIXED, "n_total"),
])
def test_create_rejects_bad_arguments(lib, bunches, n_total, state, prec, msg):
    with pytest.raises(pp.PPError) as e:
        pp.pp_create(bunches, n_total, state, prec)
    assert e.value.status == pp.PP_ERR_INVALID_ARG
    assert msg in e.value.message


def test_calls_on_null_context(lib):
    assert lib.pp_push(None, 1) == pp.PP_ERR_INVALID_ARG
    assert lib.pp_field(None, None, None, None, None) == pp.PP_ERR_INVALID_ARG
    assert lib.pp_step_batched(None, 1, 0) == pp.PP_ERR_INVALID_ARG
    assert lib.pp_diagnostics(None, None) == pp.PP_ERR_INVALID_ARG
    assert lib.pp_sync(None) == pp.PP_ERR_INVALID_ARG


def test_package_has_no_oracle_dependency():
    """The product path must not import or load the oracle."""
    pkg = os.path.join(ROOT, "paper_2502_10640_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"(import\s+oracle|from\s+oracle|libpporacle|pp_oracle|oracle_\w+\()", txt), f


def test_noalloc_rejects_bad_arguments_before_the_device(lib):
    """pp_field_noalloc checks its arguments before any device call (here
    there is no device) and reports through pp_last_error(NULL)."""
    p = 0x1000
    cases = [
        ((0, p, p, p, p, 1.0, 0.0, pp.PP_MIXED, p, p, p, None, None), "1..65536"),
        ((pp.NOALLOC_MAX_N + 1, p, p, p, p, 1.0, 0.0, pp.PP_MIXED, p, p, p, None, None), "allocation-free"),
        ((10, None, p, p, p, 1.0, 0.0, pp.PP_FP64, p, p, p, None, None), "NULL"),
        ((10, p, p, p, p, 1.0, 0.0, pp.PP_FP64, p, p, None, None, None), "NULL"),
        ((10, p, p, p, p, 0.0, 0.0, pp.PP_FP64, p, p, p, None, None), "weight > 0"),
        ((10, p, p, p, p, 1.0, float("nan"), pp.PP_FP64, p, p, p, None, None), "softening"),
        ((10, p, p, p, p, 1.0, 0.0, 9, p, p, p, None, None), "precision"),
    ]
    for args, msg in cases:
        assert lib.pp_field_noalloc(*args) == pp.PP_ERR_INVALID_ARG
        assert msg in pp.pp_last_error(None)
