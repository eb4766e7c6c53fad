"""The C-ABI library loads and exports every symbol include/nlq.h declares (no
GPU compute here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "nlq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nlq_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("nlq_assemble", "nlq_solve", "nlq_set_data", "nlq_csr_copy", "nlq_submit",
                 "nlq_wait", "nlq_pair_blocks", "nlq_mesh_box"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2101_08825_amd import nlq
    lib = ctypes.CDLL(nlq.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(nlq.EXPORTS) == _declared()


def test_errors_without_gpu_are_status_codes():
    """With no device visible, creating a context fails with a status (no abort)."""
    from paper_2101_08825_amd import nlq
    import pytest
    if os.environ.get("HIP_VISIBLE_DEVICES") is None:
        try:
            import torch
            if torch.cuda.is_available():
                pytest.skip("a GPU is present")
        except Exception:
            pass
    with pytest.raises(nlq.NlqError):
        nlq.Context(0)
    assert nlq.lib().nlq_last_error() != b""
