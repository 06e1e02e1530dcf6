"""The C-ABI library loads and exports every function include/rnsfhe.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rnsfhe.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_operations():
    names = declared_functions()
    for op in ("rf_ntt", "rf_intt", "rf_hmult_relin", "rf_rotate", "rf_rescale", "rf_modswitch",
               "rf_ctx_create", "rf_ctx_destroy", "rf_workspace_bytes", "rf_last_error"):
        assert op in names


def test_library_exports_every_declared_symbol():
    import paper_2503_22227_amd as pkg
    lib = ctypes.CDLL(pkg._lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert pkg.lib.rf_version().startswith(b"rnsfhe")


def test_binding_names_match_header():
    import paper_2503_22227_amd._lib as L
    assert set(L._SIGS) == set(declared_functions())


def test_null_arguments_fail_cleanly_without_gpu():
    import paper_2503_22227_amd._lib as L
    assert L.lib.rf_ctx_create(None, 0, None) == L.RF_EINVAL
    assert L.lib.rf_last_error() != b""
    assert L.lib.rf_ntt(None, None, 0, 1, 1, None) == L.RF_EINVAL
    assert L.lib.rf_workspace_bytes(None, 1, 1) == 0


def test_prime_chains_agree_with_oracle():
    """Both sides derive the chains independently from the same description."""
    import synthetic
    from oracle import params as OP
    from paper_2503_22227_amd import params as PP
    for name, w in synthetic.WORKLOADS.items():
        o = OP.make_params(w)
        c = PP.chain_for(w)
        assert (o.q, o.p, o.b, o.msk) == (c["q"], c["p"], c["b"], c["msk"]), name
