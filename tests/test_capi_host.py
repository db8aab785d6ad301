"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, and validates parameters before touching
the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "madlens.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


@pytest.fixture(scope="module")
def lib():
    from paper_2012_07266_amd import _lib
    return _lib.lib()


def test_header_declares_the_hot_path():
    names = _declared_functions()
    for n in ("pm_create", "pm_destroy", "pm_init_ic", "pm_step", "lens_project",
              "pm_footprint", "pm_get_state", "pm_set_state", "pm_sync", "pm_strerror"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2012_07266_amd._lib import SIGNATURES
    declared = _declared_functions()
    for n in declared:
        assert hasattr(lib, n), n
        assert n in SIGNATURES, f"{n} declared in the header but not bound"


def _params(**kw):
    from paper_2012_07266_amd.sim import make_lens, make_params
    lens_kw = {k: kw.pop(k) for k in ("npix", "fov_deg", "z_src") if k in kw}
    base = dict(np_side=32, nm_side=64, box=100.0)
    base.update(kw)
    p = make_params(**base)
    l = make_lens(lens_kw.get("npix", 64), lens_kw.get("fov_deg", 2.0),
                  lens_kw.get("z_src", (1.0,)))
    return p, l


def test_footprint(lib):
    p, l = _params(np_side=256, nm_side=512, box=205.0, npix=2048, fov_deg=5.0,
                   z_src=(0.5, 1.0, 1.5, 2.0))
    fp = lib.pm_footprint(ctypes.byref(p), ctypes.byref(l))
    # particles (2 x 28 B + 12 B acc + 8 B sort) + 3 meshes + halos, ~3.0 GB,
    # plus the reverse-pass scratch (2 x 12 B per particle + noise), ~0.47 GB
    assert 3.2e9 < fp < 3.7e9


def test_footprint_counts_the_optional_modes(lib):
    """PM_MODE_PGD adds the filter table, the shift [3][P] and one spare mesh
    with its Nyquist plane; PM_MODE_TANGENT adds 15 P values (x_dot, p_dot,
    each with the sort's second buffer, and f_dot); both add their sum;
    PM_MODE_CKPT_FORCE adds nothing to the arena."""
    from paper_2012_07266_amd._lib import PM_MODE_PGD, PM_MODE_TANGENT
    np_, nm = 128, 256
    P, es = np_ ** 3, 4
    fp = {}
    for m in (0, PM_MODE_PGD, PM_MODE_TANGENT, PM_MODE_PGD | PM_MODE_TANGENT):
        p, l = _params(np_side=np_, nm_side=nm, box=128.0, modes=m)
        fp[m] = lib.pm_footprint(ctypes.byref(p), ctypes.byref(l))
    pgd = (3 * (nm // 2) ** 2 + 1) * es + 3 * P * es + nm ** 3 * es + 2 * nm * nm * es
    tan = 15 * P * es
    slack = 5 * 256  # each buffer is 256-byte aligned
    assert 0 <= fp[PM_MODE_PGD] - fp[0] - pgd <= slack
    assert 0 <= fp[PM_MODE_TANGENT] - fp[0] - tan <= slack
    assert 0 <= fp[PM_MODE_PGD | PM_MODE_TANGENT] - fp[0] - pgd - tan <= 2 * slack
    # PM_MODE_CKPT_FORCE enlarges the caller's checkpoints, not the arena
    from paper_2012_07266_amd._lib import PM_MODE_CKPT_FORCE
    p, l = _params(np_side=np_, nm_side=nm, box=128.0, modes=PM_MODE_CKPT_FORCE)
    assert lib.pm_footprint(ctypes.byref(p), ctypes.byref(l)) == fp[0]
    p, l = _params(modes=8)  # no such mode
    assert lib.pm_footprint(ctypes.byref(p), ctypes.byref(l)) == 0


def test_device_memory_is_allocated_only_at_creation():
    """Every hipMalloc / hipFree of the simulation library sits in pm_create's
    arena set-up or the handle's destructor, or in pm_batch_create's
    parameter block and the batch's destructor (capi.cpp), or in the serving
    loop's slot management (server.cpp); no other source allocates."""
    csrc = os.path.join(ROOT, "paper_2012_07266_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        src = open(os.path.join(csrc, f)).read()
        calls = re.findall(r"\bhip(?:Malloc\w*|Free|ExtMalloc\w*)\s*\(", src)
        if f == "capi.cpp":
            # the arena and its release; the batch's block and its release
            assert len(calls) == 4, calls
            for fn in ("int create(", "~Sim()", "~Batch()"):
                assert fn in src
        elif f != "server.cpp":
            assert not calls, (f, calls)


@pytest.mark.parametrize("bad", [
    dict(np_side=30, nm_side=60),       # not a multiple of 16
    dict(np_side=32, nm_side=96),       # B = 3
    dict(np_side=80, nm_side=160),      # prime factor 5
    dict(box=-1.0),
    dict(omega_m=1.2),
    dict(fov_deg=30.0),                 # beyond the parameter table's 22 deg
    dict(npix=8),
    dict(z_src=()),
])
def test_invalid_parameters_rejected_before_allocation(lib, bad):
    from paper_2012_07266_amd._lib import PM_EINVAL
    p, l = _params(**bad)
    assert lib.pm_footprint(ctypes.byref(p), ctypes.byref(l)) == 0
    h = ctypes.c_void_p()
    assert lib.pm_create(ctypes.byref(p), ctypes.byref(l), None, ctypes.byref(h)) == PM_EINVAL
    assert not h.value


def test_null_handles(lib):
    from paper_2012_07266_amd._lib import PM_EINVAL
    assert lib.pm_destroy(None) == PM_EINVAL
    assert lib.pm_step(None, 0.1, 0.2) == PM_EINVAL
    assert lib.lens_project(None, 0.1, 0.2, None) == PM_EINVAL
    assert lib.pm_vjp_cosmo_read(None, None) == PM_EINVAL
    assert lib.pm_checkpoint_bytes(None) == 0
    assert lib.pm_checkpoint_save(None, None) == PM_EINVAL
    assert lib.pm_checkpoint_load(None, None, 0.5) == PM_EINVAL
    assert lib.pm_init_ic_jvp(None, None, 0.0, 0.0) == PM_EINVAL
    assert lib.pm_set_tangent(None, None, None, 0.0) == PM_EINVAL
    assert lib.pm_get_tangent(None, None, None, None) == PM_EINVAL
    assert lib.pm_step_jvp(None, 0.1, 0.2) == PM_EINVAL
    assert lib.lens_project_jvp(None, 0.1, 0.2, None) == PM_EINVAL
    assert lib.pm_strerror(PM_EINVAL).decode().startswith("invalid")


def test_oracle_and_product_share_no_code():
    """The oracle imports nothing from the HIP package and vice versa."""
    for d, forbidden in (("oracle", "paper_2012_07266_amd"), ("paper_2012_07266_amd", "oracle")):
        for root, _, files in os.walk(os.path.join(ROOT, d)):
            for f in files:
                if f.endswith((".py", ".hip", ".cpp", ".h")):
                    src = open(os.path.join(root, f)).read()
                    assert not re.search(rf"^\s*(from|import)\s+{forbidden}\b", src, re.M), f
