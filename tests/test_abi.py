"""The C-ABI library loads and exports every entry point include/gym.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

from conftest import ROOT


def _declared():
    src = open(os.path.join(ROOT, "include", "gym.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gym_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("gym_create", "gym_d_apply", "gym_mass_apply", "gym_op_apply", "gym_solve",
              "gym_serve_start", "gym_serve_submit", "gym_serve_poll"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2301_01753_amd import gym
    L = ctypes.CDLL(gym.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2301_01753_amd import gym
    assert sorted(gym.SIGNATURES) == _declared()
    gym.lib()  # signatures apply cleanly


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2301_01753_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
