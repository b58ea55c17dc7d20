"""Host-only checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/mhd.h declares, and validates configurations."""
import os
import re

import pytest

from paper_2511_20337_amd import mhd, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_match_binding():
    with open(os.path.join(ROOT, "include", "mhd.h")) as f:
        src = f.read()
    declared = set(re.findall(r"^\s*(?:mhd_status|void|size_t|const char\*)\s+(mhd_\w+)\s*\(",
                              src, re.M))
    assert declared == set(mhd.SYMBOLS)


def test_library_exports_every_symbol():
    L = mhd.lib()
    for name in mhd.SYMBOLS:
        assert hasattr(L, name), name


def test_init_validates_config():
    s, _ = W.turbulence_3d(8)
    ctx = mhd.mhd_init(mhd.config_from(s))
    n = 8 ** 3
    fwd = mhd.mhd_workspace_bytes(ctx)
    assert fwd >= 8 * 8 * n  # at least the stage-1 state
    assert mhd.mhd_workspace_bytes(ctx, True) >= fwd
    mhd.mhd_destroy(ctx)
    bad = [("dim", 4), ("nx", 3), ("nz", 2), ("gamma", 1.0), ("cfl", 0.0), ("cfl", float("nan")),
           ("xmax", 0.0), ("limiter", 3), ("riemann", -1), ("precision", 3), ("integrator", 2),
           ("emf", 2), ("emf", -1), ("divb", 2)]
    for field, value in bad:
        cfg = mhd.config_from(s)
        setattr(cfg, field, value)
        with pytest.raises(mhd.MHDError) as e:
            mhd.mhd_init(cfg)
        assert e.value.status == mhd.MHD_ERR_INVALID, field
    # WENO-Z runs in FP64 only
    cfg = mhd.config_from(dict(s, limiter="wenoz", precision="mixed"))
    with pytest.raises(mhd.MHDError) as e:
        mhd.mhd_init(cfg)
    assert e.value.status == mhd.MHD_ERR_INVALID
    mhd.mhd_destroy(mhd.mhd_init(mhd.config_from(dict(s, limiter="wenoz"))))
    # the UCT-HLLD average; GLM cleaning, which has no edge EMF to select
    mhd.mhd_destroy(mhd.mhd_init(mhd.config_from(dict(s, emf="uct_hlld"))))
    ctx = mhd.mhd_init(mhd.config_from(dict(s, divb="glm")))
    assert mhd.mhd_workspace_bytes(ctx) >= 9 * 8 * n  # nine-field stage-1 state
    mhd.mhd_destroy(ctx)
    with pytest.raises(mhd.MHDError) as e:
        mhd.mhd_init(mhd.config_from(dict(s, divb="glm", emf="uct_hlld")))
    assert e.value.status == mhd.MHD_ERR_INVALID
    # a 3D plane of 2^29 cells or more (the march kernels' 32-bit in-plane
    # byte offsets), and more than 4e9 cells in all
    for nx, ny, nz in ((32768, 16384, 4), (2048, 2048, 1024)):
        cfg = mhd.config_from(s)
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        with pytest.raises(mhd.MHDError) as e:
            mhd.mhd_init(cfg)
        assert e.value.status == mhd.MHD_ERR_INVALID, (nx, ny, nz)
    cfg = mhd.config_from(s)
    cfg.nx, cfg.ny, cfg.nz = 16384, 16384, 4  # 2^28 cells per plane: accepted
    mhd.mhd_destroy(mhd.mhd_init(cfg))
    s2, _ = W.orszag_tang_2d(8)
    cfg = mhd.config_from(s2)
    cfg.nz = 4  # 2D needs nz == 1
    with pytest.raises(mhd.MHDError):
        mhd.mhd_init(cfg)
    mhd.mhd_destroy(mhd.mhd_init(mhd.config_from(s2)))


def test_strerror_texts():
    assert mhd.strerror(0) == "ok"
    assert "unphysical" in mhd.strerror(-4)
    assert "workspace" in mhd.strerror(-5)


def test_c_abi_program_rejects_bad_input_without_a_gpu(tmp_path):
    """The host program built on the bare C ABI (tests/c_abi) stops with a
    usage error for a wrong argument count and with mhd_init's status for an
    invalid configuration, both before any device call."""
    import subprocess
    exe = os.path.join(ROOT, "tests", "c_abi", "step_cli")
    assert os.path.exists(exe), "tests/c_abi/step_cli is missing: run __graft_entry__.build()"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr
    fin = tmp_path / "in.bin"
    fin.write_bytes(b"")
    bad = ["4", "8", "8", "8", "0", "1", "0", "1", "0", "1", "1.6666666666666667", "0.3",
           "1", "0", "0", "0"]  # dim 4
    r = subprocess.run([exe, str(fin), str(tmp_path / "out.bin"), "1"] + bad,
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "mhd_init" in r.stderr, r.stderr
