"""The C-ABI library loads on a host without a GPU and exports every call
that include/ks.h declares (no compute call is made here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ks.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ks_[a-z_]+)\s*\(", text)))


def test_header_declares_the_path():
    syms = declared_symbols()
    for name in ["ks_ntt", "ks_intt", "ks_bconv", "ks_modup", "ks_keymult", "ks_moddown", "ks_keyswitch",
                 "ks_params_create", "ks_params_destroy", "ks_workspace_bytes", "ks_strerror"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    # the release library and its debug twin (canonical-input checks)
    for name in ("libks.so", "libks_debug.so"):
        lib = ctypes.CDLL(os.path.join(ROOT, "paper_2603_16692_amd", name))
        missing = [s for s in declared_symbols() if not hasattr(lib, s)]
        assert not missing, (name, missing)


def test_binding_loads_and_lists_exports():
    import paper_2603_16692_amd as k
    assert set(k.EXPORTED) <= set(declared_symbols())
    assert k.raw_call("ks_strerror", 0) == b"ok"
    assert k.raw_call("ks_strerror", k.KS_EALIGN) == b"pointer not 256-byte aligned"


def test_binding_structs_match_the_header():
    # the ctypes mirrors of ks_plan and ks_info list the header's fields in order
    import paper_2603_16692_amd as k
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "ks.h")).read(), flags=re.S)
    structs = {name: body for body, name in re.findall(r"typedef struct \{([^{}]*)\}\s*(\w+);", text)}
    for cname, pycls in (("ks_plan", k.Plan), ("ks_info", k.Info)):
        fields = []
        for decl in structs[cname].split(";"):
            decl = decl.strip()
            if decl:
                fields += [re.sub(r"\[.*\]", "", n).strip() for n in decl.split(None, 1)[1].split(",")]
        assert fields == [f[0] for f in pycls._fields_], (cname, fields)
