"""The C-ABI library loads, exports every declared symbol and rejects bad arguments.

No compute call reaches a GPU here: argument validation runs before any HIP
call, so these tests run on a machine without a GPU.
"""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2111_14999_amd as pg
from paper_2111_14999_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "phoebe_gpu.h")).read()
    return sorted(set(re.findall(r"\b(phoebe_gpu_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(binding.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = pg.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.phoebe_gpu_abi_version() == 2


def test_null_handle_and_create_errors():
    lib = pg.load()
    assert lib.phoebe_gpu_create(0, 0, None) == -1
    assert b"NULL" in lib.phoebe_gpu_last_error(None)
    assert lib.phoebe_gpu_destroy(None) == 0
    assert lib.phoebe_gpu_scatter_rates(None, None, None, None, None, 0, None, None, None, None,
                                        0, None, None, None, None, None) == -1
    assert lib.phoebe_gpu_phonon_linewidth(None, None, None, None, None, 0, None, None, None,
                                           None) == -1
    assert lib.phoebe_gpu_interp_v3(None, None, None, 0, None, 0, 0.0, None, None, None, None,
                                    None) == -1
    assert lib.phoebe_gpu_philox_uniform(None, 1, 0, 4, None, None) == -1
    assert lib.phoebe_gpu_training_set(None, None, None, 0, 1, 1, 0.0, 0.0, 1, 0, None, None,
                                       None, None, 0, None, None, None) == -1
    assert lib.phoebe_gpu_set_check_finite(None, 1) == -1
    assert lib.phoebe_gpu_interp_g(None, None, None, 0, None, 0, 0.0, 0, None, None, None,
                                   None, None) == -1
    assert lib.phoebe_gpu_set_timing(None, 1) == -1
