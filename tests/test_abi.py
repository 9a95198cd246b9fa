"""The C-ABI library loads and exports every function the public header
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os

import pytest

from paper_1801_03690_amd import binding


def test_header_declares_the_boundary():
    names = binding.header_symbols()
    for required in ("mm_create", "mm_destroy", "mm_mesh_upload", "mm_material_set", "mm_energy_grad",
                     "mm_precondition", "mm_ncg_minimize", "mm_demag_curve", "mm_last_error"):
        assert required in names


def test_library_exports_every_header_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmmncg.so is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in binding.header_symbols() if not hasattr(L, n)]
    assert not missing, missing


def test_opts_defaults_without_gpu():
    o = binding.default_opts()
    assert o.jmax == 4 and o.tol_torque == 1e-6 and o.poisson_rtol == 1e-10
    assert o.theta_max == 0.2 and o.c1 == 1e-4 and o.c2 == 0.1 and o.max_nli == 20000
    assert o.poisson_prec == binding.MM_PREC_JACOBI and o.beta == binding.MM_BETA_ZA
    assert o.prec_form == binding.MM_PFORM_PAPER
    # the last fields: their values also check that the ctypes layout matches the C struct
    assert o.theta_adapt == 0 and o.theta_hi == 1.5707963267948966


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = binding.lib().mm_create(ctypes.byref(h), 0, None, binding.ALLOC_FN(), binding.FREE_FN(), None)
    assert rc == binding.MM_EDEVICE and not h.value
