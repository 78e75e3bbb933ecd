"""CPU-side checks of the C-ABI library: it loads and exports every symbol
that include/dmcx.h declares (no compute calls; no GPU needed)."""
import ctypes
import os
import re

from paper_2504_07948_amd import dmcx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "dmcx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmcx_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_expected_calls():
    names = _declared()
    for n in ["dmcx_create", "dmcx_eval_orbitals", "dmcx_ratio_grad", "dmcx_accept",
              "dmcx_flush", "dmcx_run", "dmcx_measure", "dmcx_ion_grads", "dmcx_logpsi_vjp"]:
        assert n in names
    assert set(names) == set(dmcx.EXPORTED)
    # the binding carries a function of the same name for every entry point
    missing = [n for n in names if not callable(getattr(dmcx, n, None))]
    assert not missing, missing


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(dmcx.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_loads_and_strerror():
    lib = dmcx.load()
    assert dmcx.dmcx_strerror(dmcx.DMCX_OK) == "ok"
    assert "singular" in dmcx.dmcx_strerror(dmcx.DMCX_E_SINGULAR)
    assert lib is dmcx.load()


def test_invalid_arguments_rejected_without_device():
    lib = dmcx.load()
    # NULL handles / pointers are rejected before any HIP call
    assert lib.dmcx_run(None, 1, 1, 0.0, None, None, 0) == dmcx.DMCX_E_INVALID
    assert lib.dmcx_measure(None, None, None, None, 0) == dmcx.DMCX_E_INVALID
    assert lib.dmcx_create(None, 1, None, None, None, None) == dmcx.DMCX_E_INVALID


def test_sweep_traffic_hash_covers_the_compiler_flags():
    """The sweep's stored traffic figures are keyed by a hash of its sources
    and of the flags it is compiled with: a change of either invalidates
    them."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    from paper_2504_07948_amd import build_ext
    h0 = bench.kernel_sources_sha256()
    saved = dict(build_ext.SOURCE_FLAGS)
    try:
        build_ext.SOURCE_FLAGS["sweep_f64.hip"] = saved.get("sweep_f64.hip", []) + ["-DX"]
        assert bench.kernel_sources_sha256() != h0
        build_ext.SOURCE_FLAGS.pop("sweep_f64.hip")
        assert bench.kernel_sources_sha256() != h0 or not saved.get("sweep_f64.hip")
    finally:
        build_ext.SOURCE_FLAGS.clear()
        build_ext.SOURCE_FLAGS.update(saved)
    assert bench.kernel_sources_sha256() == h0
