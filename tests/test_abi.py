"""The C-ABI library loads on a machine without a GPU and exports every function
that include/fam.h declares; status strings and error paths that need no device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2609_26194_amd import fam
    if not os.path.exists(fam.LIB_PATH):
        from paper_2609_26194_amd.build import build
        build()
    return fam.load_library()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fam.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fam_\w+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("fam_init", "fam_init_batched", "fam_step", "fam_run", "fam_adjoint", "fam_stage", "fam_oe",
              "fam_dt", "fam_check", "fam_destroy", "fam_state_len", "fam_status_str"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    lib = _lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert len(lib.fam_status_str(code)) > 0


def test_invalid_configurations_are_rejected_without_a_device():
    from paper_2609_26194_amd.fam import FAM_ERR_ARG, FAM_ERR_SIZE, FamConfig
    lib = _lib()
    h = ctypes.c_void_p()
    for bad in (dict(dim=3, nx=8, ny=8), dict(dim=2, nx=8, ny=8, k=7), dict(dim=2, nx=2, ny=8),
                dict(dim=2, nx=8, ny=8, cfl=0.0), dict(dim=2, nx=8, ny=8, gamma=1.0),
                dict(dim=2, nx=8, ny=8, x0=1.0, x1=0.0), dict(dim=2, nx=65536, ny=32769),
                dict(dim=1, nx=2), dict(dim=1, nx=8, pp=True), dict(dim=2, nx=8, ny=8, system="advection", dmr=True),
                dict(dim=1, nx=8, system="euler", dmr=True), dict(dim=2, nx=8, ny=8, dt_rule=2),
                dict(dim=2, nx=8, ny=8, k=4, char_vars=True), dict(dim=1, nx=8, system="burgers", char_vars=True)):
        cfg = FamConfig(**bad)
        assert lib.fam_init(ctypes.byref(cfg.to_c()), None, ctypes.byref(h)) == FAM_ERR_ARG
    # enum values outside their range
    for field, value in (("oe", 3), ("bc_x", 2), ("bc_y", -1), ("system", 3)):
        c = FamConfig(dim=2, nx=8, ny=8).to_c()
        setattr(c, field, value)
        assert lib.fam_init(ctypes.byref(c), None, ctypes.byref(h)) == FAM_ERR_ARG
    assert lib.fam_init(None, None, ctypes.byref(h)) == FAM_ERR_ARG
    # batched contexts: OE Type I and the double Mach reflection boundaries are single-context options
    for extra in (dict(oe="type1"), dict(system="euler", dmr=True, x1=3.0), dict(system="euler", char_vars=True)):
        arr = (type(FamConfig(dim=2, nx=8, ny=8).to_c()) * 2)(*[FamConfig(dim=2, nx=8, ny=8, **extra).to_c()] * 2)
        assert lib.fam_init_batched(arr, 2, None, ctypes.byref(h)) == FAM_ERR_ARG
    assert lib.fam_step(None, None, 0.0, None) == FAM_ERR_ARG
    assert lib.fam_run(None, None, 1.0, 0, 0.0, None, None) == FAM_ERR_ARG
    assert lib.fam_set_time(None, 0.0) == FAM_ERR_ARG
    # the allocation-free step: argument checks and the size limit come before any device work
    ok = FamConfig(dim=2, nx=64, ny=64, system="euler").to_c()
    fake = ctypes.c_void_p(256)
    assert lib.fam_step_static(None, None, fake, 0.0, 0.0, None, None) == FAM_ERR_ARG
    assert lib.fam_step_static(ctypes.byref(ok), None, None, 0.0, 0.0, None, None) == FAM_ERR_ARG
    assert lib.fam_step_static(ctypes.byref(ok), None, fake, float("nan"), 0.0, None, None) == FAM_ERR_ARG
    big = FamConfig(dim=2, nx=600, ny=600, system="euler").to_c()    # 4.3e6 doubles: more than 64 MiB holds
    assert lib.fam_step_static(ctypes.byref(big), None, fake, 0.0, 0.0, None, None) == FAM_ERR_SIZE
    assert lib.fam_dbg_recon(None, None, None) == FAM_ERR_ARG
    assert lib.fam_dbg_oe_factors(None, None, None, None) == FAM_ERR_ARG


def test_binding_rejects_wrong_sized_states():
    """The wrapper checks sizes before any launch (no GPU needed for the check itself)."""
    import torch
    from paper_2609_26194_amd.fam import Fam
    fake = Fam.__new__(Fam)
    fake.len = 10
    fake.cfgs = [None]
    with pytest.raises(ValueError):
        fake._state(torch.zeros(11, dtype=torch.float64))


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback path: without libfam.so the binding raises before any computation."""
    from paper_2609_26194_amd import fam
    monkeypatch.setattr(fam, "_lib", None)
    monkeypatch.setattr(fam, "LIB_PATH", str(tmp_path / "libfam.so"))
    with pytest.raises(RuntimeError, match="missing"):
        fam.load_library()
    # the context raises too (here first for the missing device, on a machine with a GPU for the library)
    with pytest.raises(RuntimeError):
        fam.Fam(fam.FamConfig(dim=2, nx=8, ny=8))


def test_ctypes_config_mirrors_the_header():
    """The binding's fam_config has the header's fields, in the header's order."""
    from paper_2609_26194_amd.fam import _CConfig
    text = open(os.path.join(ROOT, "include", "fam.h")).read()
    body = re.sub(r"/\*.*?\*/", "", text.split("typedef struct {", 1)[1].split("} fam_config;", 1)[0], flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            fields += [n.strip() for n in decl.split(None, 1)[1].split(",")]
    assert [f for f, _ in _CConfig._fields_] == fields
