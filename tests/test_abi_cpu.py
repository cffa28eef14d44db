"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kpm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kpm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1410_5242_amd import kpm
    if not os.path.exists(kpm.LIB_PATH):
        pytest.skip("libkpm.so not built (run __graft_entry__.build())")
    return kpm.lib()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("kpm_build_hamiltonian", "kpm_moments", "kpm_dos", "kpm_aug_spmmv",
              "kpm_export_csr", "kpm_hamiltonian_info", "kpm_destroy_hamiltonian",
              "kpm_last_error", "kpm_version"):
        assert s in syms


def test_library_exports_every_declared_symbol(L):
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_1410_5242_amd", "libkpm.so"))
    for s in declared_symbols():
        assert hasattr(raw, s), s


def test_version_and_error_strings(L):
    assert b"gfx950" in L.kpm_version()
    assert isinstance(L.kpm_last_error(), bytes)


def test_argument_validation_without_device(L):
    from paper_1410_5242_amd import kpm
    out = ctypes.c_void_p(1)
    assert L.kpm_build_hamiltonian(None, None, ctypes.byref(out)) == kpm.KPM_EINVAL
    assert out.value is None
    assert b"desc" in L.kpm_last_error()
    d = kpm.LatticeDesc()
    d.L[0] = d.L[1] = d.L[2] = 4
    d.periodic[0] = d.periodic[1] = d.periodic[2] = 1
    d.t, d.margin = 1.0, 1.01
    d.gamma = -1.0   # no potential array: the generated one needs a finite gamma >= 0
    assert L.kpm_build_hamiltonian(ctypes.byref(d), None, ctypes.byref(out)) == kpm.KPM_EINVAL
    assert b"gamma" in L.kpm_last_error()
    d.gamma = float("nan")
    assert L.kpm_build_hamiltonian(ctypes.byref(d), None, ctypes.byref(out)) == kpm.KPM_EINVAL
    fake = ctypes.c_void_p(0x1000)
    assert L.kpm_moments(None, fake, 1, 8, fake, None, None) == kpm.KPM_EINVAL
    opts = kpm.RunOpts()
    opts.variant = kpm.PLAIN   # moments run the FULL or NODOT variant
    assert L.kpm_moments(fake, fake, 1, 8, fake, ctypes.byref(opts), None) == kpm.KPM_EINVAL
    opts.variant = kpm.FULL
    assert L.kpm_moments(fake, fake, 1, 7, fake, ctypes.byref(opts), None) == kpm.KPM_EINVAL      # odd M
    assert L.kpm_moments(fake, fake, 3, 8, fake, ctypes.byref(opts), None) == kpm.KPM_ENOTSUP     # R
    assert L.kpm_moments(fake, ctypes.c_void_p(0x1008), 1, 8, fake, ctypes.byref(opts), None) == kpm.KPM_EINVAL
    bad = kpm.SweepTuning(*[0] * 12)
    bad.prefetch = 9
    opts.tuning = ctypes.pointer(bad)   # a per-call tuning is validated like kpm_set_sweep_tuning
    assert L.kpm_moments(fake, fake, 1, 8, fake, ctypes.byref(opts), None) == kpm.KPM_EINVAL
    assert L.kpm_set_sweep_tuning(ctypes.byref(bad)) == kpm.KPM_EINVAL
    plan = kpm.SweepPlan()
    assert L.kpm_sweep_plan(None, 32, None, ctypes.byref(plan)) == kpm.KPM_EINVAL
    assert L.kpm_aug_spmmv(None, fake, fake, 1, 1.0, 0.0, 0.0, 0, None, None) == kpm.KPM_EINVAL
    assert L.kpm_dos(None, 1, 8, 0, 0.0, 1.0, 0.0, fake, 4, fake, None) == kpm.KPM_EINVAL
    assert L.kpm_dos(fake, 1, 8, 0, 0.0, 1.0, 0.0, fake, 0, fake, None) == kpm.KPM_EINVAL   # K = 0
    assert L.kpm_dos(fake, 1, 8, 0, 0.0, -1.0, 0.0, fake, 4, fake, None) == kpm.KPM_EINVAL  # a <= 0
    assert L.kpm_dos(fake, 1, 8, 7, 0.0, 1.0, 0.0, fake, 4, fake, None) == kpm.KPM_EINVAL   # kernel
    assert L.kpm_dos(fake, 1, 8, 2, 0.0, 1.0, 0.0, fake, 4, fake, None) == kpm.KPM_EINVAL   # Lorentz lambda
    assert L.kpm_hamiltonian_info(None, None, None, None, None, None, None, None, None) == kpm.KPM_EINVAL
    assert L.kpm_moments_naive(None, fake, 1, 8, fake, 0, None) == kpm.KPM_EINVAL
    assert L.kpm_axpy(7, 4, 1.0, fake, fake, None) == kpm.KPM_EINVAL                  # dtype
    assert L.kpm_axpy(0, -1, 1.0, fake, fake, None) == kpm.KPM_EINVAL                 # n < 0
    assert L.kpm_axpy(0, 4, 1.0, ctypes.c_void_p(0x1008), fake, None) == kpm.KPM_EINVAL  # misaligned
    assert L.kpm_scal(1, 4, 1.0, None, None) == kpm.KPM_EINVAL                        # NULL vector
    assert L.kpm_dot(0, 4, fake, fake, None, None) == kpm.KPM_EINVAL                  # NULL out
    assert L.kpm_axpy(0, 0, 1.0, None, None, None) == kpm.KPM_OK                      # empty: no-op
    lo, hi = ctypes.c_double(), ctypes.c_double()
    assert L.kpm_lanczos_bounds(None, 10, 0, ctypes.byref(lo), ctypes.byref(hi), None) == kpm.KPM_EINVAL
    assert L.kpm_set_scaling(None, 1.0, 0.0) == kpm.KPM_EINVAL
    assert L.kpm_site_block(None, 4, 1, fake, 0, None) == kpm.KPM_EINVAL
    assert L.kpm_plane_wave_block(fake, None, 1, fake, fake, 0, None) == kpm.KPM_EINVAL
    assert L.kpm_sweep_profile_enable(-1) == kpm.KPM_EINVAL   # sampling period < 0
    assert L.kpm_sweep_profile_enable(0) == kpm.KPM_OK
    L.kpm_destroy_hamiltonian(None)   # no-op


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1410_5242_amd import kpm
    monkeypatch.setattr(kpm, "_LIB", None)
    monkeypatch.setattr(kpm, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        kpm.lib()


def test_struct_layouts_match_the_header():
    # the ctypes mirrors of the header's structs: field names in header order
    from paper_1410_5242_amd import kpm
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)

    def fields(struct_end):
        body = re.search(r"typedef struct[^{]*\{([^}]*)\}\s*" + struct_end + r"\s*;", text).group(1)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            for part in decl.split(","):
                m = re.search(r"([A-Za-z_][A-Za-z_0-9]*)\s*(\[\d+\])?\s*$", part.strip())
                names.append(m.group(1))
        return names

    for cls, name in ((kpm.LatticeDesc, "kpm_lattice_desc"), (kpm.RunOpts, "kpm_run_opts"),
                      (kpm.SweepTuning, "kpm_sweep_tuning"), (kpm.BatchTuning, "kpm_batch_tuning"),
                      (kpm.SweepPlan, "kpm_sweep_plan_info"), (kpm.CsrDesc, "kpm_csr_desc")):
        assert [f[0] for f in cls._fields_] == fields(name), name
