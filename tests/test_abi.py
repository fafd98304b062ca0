"""The C-ABI library loads and exports every entry point include/newmark.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "newmark.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("nm_newmark_init", "nm_newmark_step", "nm_apply_operator", "nm_precond_apply"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2211_08263_amd import newmark
    if not os.path.exists(newmark.LIB_PATH):
        pytest.skip("libnewmark.so not built")
    lib = ctypes.CDLL(newmark.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(newmark.EXPORTED) == set(_declared())


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    from paper_2211_08263_amd import newmark
    monkeypatch.setattr(newmark, "_lib", None)
    monkeypatch.setattr(newmark, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        newmark.load_library()


def test_library_shares_the_hip_runtime_of_torch():
    """One HIP runtime per process: the library binds to the one PyTorch loaded."""
    from paper_2211_08263_amd import newmark as nmb
    nmb.load_library()
    rts = nmb.hip_runtimes_loaded()
    assert len(rts) == 1, rts


def _bad_init(**change):
    """nm_newmark_init on a small valid problem with one argument made invalid; every check
    below fails before any device work, so these run without a GPU."""
    import numpy as np
    from paper_2211_08263_amd import newmark as nmb
    from paper_2211_08263_amd import workloads as W
    pb = W.make_polycrystal(n=16, n_grains=4, seed=1)
    args = dict(dim=3, n=pb.n, L=pb.L, phase_id=pb.phase_id, C_voigt=pb.C21, rho=pb.rho, gamma_idx=pb.gamma_idx,
                dt=pb.dt, options=nmb.Options())
    args.update(change)
    with pytest.raises(nmb.NewmarkError) as e:
        nmb.newmark_init(**args)
    return e.value.code


@pytest.mark.parametrize("case,code", [
    ("grid not a power of two", "EUNSUPPORTED"),
    ("axis above 512", "EUNSUPPORTED"),
    ("dim 4", "EUNSUPPORTED"),
    ("2D with n3 > 1", "EUNSUPPORTED"),
    ("duplicate Gamma index", "EINVAL"),
    ("unsorted Gamma", "EINVAL"),
    ("Gamma index out of range", "EINVAL"),
    ("phase id out of range", "EINVAL"),
    ("non-positive density", "EINVAL"),
    ("non-positive dt", "EINVAL"),
    ("non-positive tol", "EINVAL"),
    ("unknown warm start", "EINVAL"),
    ("negative damping", "EINVAL"),
    ("non-finite damping", "EINVAL"),
    ("damping in the explicit scheme", "EUNSUPPORTED"),
    ("unknown differentiation rule", "EINVAL"),
])
def test_init_rejects_bad_arguments(case, code):
    import numpy as np
    from paper_2211_08263_amd import newmark as nmb
    from paper_2211_08263_amd import workloads as W
    pb = W.make_polycrystal(n=16, n_grains=4, seed=1)
    g = pb.gamma_idx
    change = {
        "grid not a power of two": dict(n=(96, 16, 16), phase_id=np.zeros((16, 16, 96), np.uint16)),
        "axis above 512": dict(n=(1024, 16, 16), phase_id=np.zeros((16, 16, 1024), np.uint16)),
        "dim 4": dict(dim=4),
        "2D with n3 > 1": dict(dim=2),
        "duplicate Gamma index": dict(gamma_idx=np.concatenate([g[:3], g[2:3], g[3:]])),
        "unsorted Gamma": dict(gamma_idx=g[::-1].copy()),
        "Gamma index out of range": dict(gamma_idx=np.array([0, 16 ** 3], np.int64)),
        "phase id out of range": dict(phase_id=np.full(pb.phase_id.shape, 7, np.uint16)),
        "non-positive density": dict(rho=np.array([1.0, 0.0, 1.0, 1.0])),
        "non-positive dt": dict(dt=0.0),
        "non-positive tol": dict(options=nmb.Options(tol=0.0)),
        "unknown warm start": dict(options=nmb.Options(warm_start=9)),
        "negative damping": dict(damping=np.array([0.0, -1.0, 0.0, 0.0])),
        "non-finite damping": dict(damping=np.array([0.0, np.nan, 0.0, 0.0])),
        "damping in the explicit scheme": dict(damping=np.array([0.0, 1.0, 0.0, 0.0]), beta=0.0),
        "unknown differentiation rule": dict(diff_rule=3),
    }[case]
    assert _bad_init(**change) == getattr(nmb, "NM_" + code)
