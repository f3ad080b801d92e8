"""The C-ABI library loads and exports every entry point include/rb.h
declares; the Python binding names match (no GPU needed, no compute call)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(rb_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rb_create", "rb_tree_build", "rb_gravity", "rb_step", "rb_tree_export",
                 "rb_batch_create", "rb_batch_step", "rb_state_save", "rb_state_load",
                 "rb_destroy", "rb_error_string", "rb_direct"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1110_4876_amd import rb
    L = rb.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1110_4876_amd import rb
    assert set(_declared()) == set(rb._SIGS)


def test_error_strings_without_gpu():
    from paper_1110_4876_amd import rb
    assert rb.rb_error_string(rb.RB_EINVAL) == "invalid argument"
    assert rb.rb_error_string(rb.RB_ECAPACITY) == "capacity exceeded"
    p = rb.params()
    assert p.theta == 0.5 and p.leaf_size == 1 and p.group_size == 64
