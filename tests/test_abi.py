"""The C-ABI library loads and exports every symbol include/cpm.h declares (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2201_12963_amd", "libcpm.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("cpm_create", "cpm_build_elastance", "cpm_solve", "cpm_solve_batch", "cpm_grad",
              "cpm_get_matrix", "cpm_last_error", "cpm_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpm.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (one HIP runtime per process: torch's)
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n
    from paper_2201_12963_amd import binding
    assert set(binding.EXPORTED) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcpm.so not built")
def test_create_rejects_bad_descriptors_without_gpu():
    """Descriptor validation, mesh factorisation and LDS sizing included,
    happens before any device call."""
    import numpy as np
    from paper_2201_12963_amd import binding
    from workloads import make_workload
    w = make_workload("tiny", "ff")
    base = dict(box=w.box, geometry=0, kspace=0, precision=0, eta=w.eta, alpha=w.alpha, rcut=w.rcut,
                kcut=w.kcut, mesh=w.mesh, order=w.order, alpha_build=w.alpha_exact, rcut_build=w.rcut_exact,
                kcut_build=w.kcut_exact, elec_xyz=w.elec_xyz, elec_side=w.elec_side, elec_sub=None,
                site_q=w.site_q)
    cases = [
        dict(alpha=w.eta),                                  # alpha >= eta / sqrt 2
        dict(box=np.array([1.0, -1.0, 1.0])),
        dict(site_q=w.site_q + 0.01),                        # not neutral
        dict(elec_side=np.zeros(w.n_elec, np.int8)),
        dict(geometry=1),                                    # doubled cell without elec_sub
        dict(kspace=1, mesh=(16, 4, 64), order=5),           # fewer mesh points than the stencil
        dict(kspace=1, mesh=(7, 16, 64)),                    # 7 is not a product of 2, 3 and 5
        dict(kspace=1, mesh=(16, 16, 4096)),                 # longer z columns than the z pass takes
        dict(kspace=1, mesh=(64, 64, 64)),                   # FP64 plane + staging list exceed LDS
        dict(kspace=0, precision=1),                         # mixed precision needs PPPM
    ]
    for over in cases:
        with pytest.raises(binding.CpmError) as ei:
            binding.Context(**{**base, **over})
        assert ei.value.code == binding.CPM_EINVAL
