"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every symbol the
header declares, derives the paper's parameters like the oracle does, and rejects bad arguments
before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lbm():
    import paper_1308_2071_amd as m
    m.library()
    return m


def header_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lbm):
    from paper_1308_2071_amd import _abi
    names = header_functions()
    assert len(names) >= 18
    lib = C.CDLL(_abi.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.EXPORTED)


def test_param_struct_layout_matches_header(lbm, tmp_path):
    """The ctypes mirrors have the layout the C compiler gives the header's structs: every
    field's offset and the sizes, printed by a program compiled against include/lbm.h."""
    import subprocess
    from paper_1308_2071_amd._abi import LbmObs, LbmParams
    structs = {"lbm_params": LbmParams, "lbm_obs": LbmObs}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', "int main(void) {"]
    for cname, py in structs.items():
        src.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            src.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    src.append("return 0; }")
    (tmp_path / "layout.c").write_text("\n".join(src))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c11", "-I", inc, "-o", str(exe),
                           str(tmp_path / "layout.c")])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out.splitlines()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_defaults_are_the_papers(lbm):
    p = lbm.lbm_default_params()
    assert (p.rho0, p.varpi, p.J, p.sigma, p.Ma) == (1.0, -2.0, 1.0, 1.0, 0.1)
    assert (p.s_e, p.s_eps, p.s_q, p.zeta3, p.zeta4) == (1.1, 1.1, 1.2, 1.5, 1.5)
    assert tuple(p.bc) == (0, 0, 1, 1)
    assert tuple(p.T_wall)[:2] == (1.0, 0.0)


@pytest.mark.parametrize("case", [
    dict(nx=64, ny=64, Ra=1e3, Pr=1.0, Da=1e-2),
    dict(nx=256, ny=256, Ra=1e5, Pr=1.0, Da=1e-2),
    dict(nx=4096, ny=4096, Ra=1e6, Pr=0.71, Da=1e-3),
    dict(nx=100, ny=37, Ra=3e4, Pr=7.0, Da=-1.0, J=1.3, sigma=0.8, varpi=-1.0),
    dict(nx=151, ny=151, Ra=1e5, Ra_I=1e3, Pr=0.7, Da=1e-2),
    dict(nx=121, ny=121, Ra=0.0, Ra_I=6.4e5, Pr=7.0, bc=(0, 0, 0, 0), T_wall=(0.0, 0.0, 0.0, 0.0),
         T_init=0.0, forchheimer=0, Da=-1.0),
    dict(nx=20, ny=9, Ra=1e4, Qv=3e-5, sigma=1.2),
])
def test_derived_parameters_match_oracle(lbm, oracle, case):
    d = lbm.lbm_derived(lbm.make_params(**case))
    r = oracle.derived(**case)
    for k in ("L", "tau_v", "tau_T", "nu_e", "nu", "gbeta", "dT", "T0", "Q"):
        assert d[k] == pytest.approx(r[k], rel=1e-14), k
    assert d["K"] == pytest.approx(r["K_uniform"], rel=1e-14) or (np.isinf(d["K"]) and
                                                                   np.isinf(r["K_uniform"]))


def status_of(lbm, **kw):
    from paper_1308_2071_amd import _abi
    p = lbm.make_params(**kw)
    n = C.c_size_t()
    return _abi.library().lbm_workspace_size(C.byref(p), 100, C.byref(n))


@pytest.mark.parametrize("bad", [
    dict(nx=4),                                  # five-point stencil needs 5 nodes
    dict(ny=3),
    dict(bc=(2, 0, 1, 1)),                       # unpaired periodic side
    dict(bc=(0, 0, 2, 1)),
    dict(bc=(0, 0, 1, 7)),                       # unknown side condition
    dict(varpi=1.0),                             # Eq. (29): varpi < 1
    dict(rho0=0.0),
    dict(sigma=-1.0),
    dict(tau_v=0.5),                             # tau must exceed 1/2
    dict(tau_T=0.4),
    dict(Ra=-1.0),
    dict(Ra=0.0),                                # neither Ra nor Ra_I
    dict(Ra_I=-5.0),
    dict(dtype=5),
    dict(s_q=2.5),
    dict(checkpoint_every=-3),
    dict(nx=40000, ny=40000),                    # beyond the 2^31-element state limit
])
def test_invalid_parameters_are_rejected(lbm, bad):
    assert status_of(lbm, **bad) == -1  # LBM_E_INVAL
    assert lbm.lbm_last_error() != ""


def test_state_limit_is_exact(lbm):
    """The 2^31-element state limit counts the 14 planes as they lie in memory: ny rows of the
    pitch (nx rounded up to 64) plus the pad between planes.  12354^2 (pitch 12416, 14 x
    (12416 x 12354 + 1056) = 2,147,436,480 elements) is the largest square grid under it."""
    assert status_of(lbm, nx=12354, ny=12354, dtype=1) == 0
    assert status_of(lbm, nx=12355, ny=12355, dtype=1) == -1


def test_init_rejects_before_any_device_call(lbm):
    from paper_1308_2071_amd import _abi
    L = _abi.library()
    p = lbm.make_params(nx=16, ny=16)
    h = C.c_void_p()
    # null workspace
    assert L.lbm_init(C.byref(h), C.byref(p), None, None, 0.5, None, 1 << 20, None) == -1
    # phi_uniform outside (0, 1]
    assert L.lbm_init(C.byref(h), C.byref(p), None, None, 1.5, 256, 1 << 20, None) == -1
    # misaligned workspace
    assert L.lbm_init(C.byref(h), C.byref(p), None, None, 0.5, 8, 1 << 20, None) == -1
    # too small workspace (no device call either)
    assert L.lbm_init(C.byref(h), C.byref(p), None, None, 0.5, 256, 64, None) == -2
    assert h.value is None


def test_null_context_and_status_strings(lbm):
    from paper_1308_2071_amd import _abi
    L = _abi.library()
    assert L.lbm_step(None, 1) == -1
    assert L.lbm_grad(None, 1.0, None, None) == -1
    assert L.lbm_destroy(None) == 0
    for s, name in [(0, "LBM_OK"), (-1, "LBM_E_INVAL"), (-4, "LBM_E_DIVERGED"),
                    (-6, "LBM_E_UNSUPPORTED"), (17, "LBM_E_UNKNOWN")]:
        assert lbm.lbm_status_string(s) == name


def test_workspace_grows_with_tape(lbm):
    base = lbm.lbm_workspace_size(lbm.make_params(nx=64, ny=64), 0)
    tape = lbm.lbm_workspace_size(lbm.make_params(nx=64, ny=64, checkpoint_every=100), 2000)
    state = 14 * 64 * 64 * 4
    assert base >= 2 * state
    # 20 checkpoints + two banks of 100 segment states + 2 adjoint buffers
    assert tape - base >= (20 + 200 + 2) * state


def test_aa_layout_halves_the_state_memory(lbm):
    pull = lbm.lbm_workspace_size(lbm.make_params(nx=300, ny=200), 0)
    aa = lbm.lbm_workspace_size(lbm.make_params(nx=300, ny=200, layout="aa"), 0)
    # pitch 320 = 300 rounded up to 64; the planes lie 200 rows plus a pad of 1056 elements apart
    state = 14 * (200 * 320 + 1056) * 4
    assert pull - aa == state


def test_aa_layout_limits(lbm):
    assert status_of(lbm, layout=3) == -1                          # LBM_E_INVAL
    assert status_of(lbm, steps_per_launch=4) == 0                 # 16 x 16 tiles in LDS
    assert status_of(lbm, steps_per_launch=8) == 0                 # 8 x 8 tiles in LDS
    assert status_of(lbm, steps_per_launch=5) == -1
    assert status_of(lbm, steps_per_launch=6) == -1
    assert status_of(lbm, layout=1, checkpoint_every=10) == -6     # LBM_E_UNSUPPORTED: no tape
    from paper_1308_2071_amd import _abi
    p = (_abi.LbmParams * 1)(lbm.make_params(nx=16, ny=16, layout="aa"))
    n = C.c_size_t()
    assert _abi.library().lbm_batch_workspace_size(1, p, C.byref(n)) == -6


def test_three_steps_per_launch_need_fp32_and_a_state_below_2_gib(lbm):
    assert status_of(lbm, steps_per_launch=3) == 0
    assert status_of(lbm, dtype=1, steps_per_launch=3) == -6       # FP64: LBM_E_UNSUPPORTED
    assert status_of(lbm, dtype=2, steps_per_launch=3) == -6       # FP32 storage, FP64 arithmetic
    # 14 planes of pitch x ny + 1056 FP32 elements: 6100^2 holds 2.10e9 bytes, 6200^2 2.16e9
    assert status_of(lbm, nx=6100, ny=6100, steps_per_launch=3) == 0
    assert status_of(lbm, nx=6200, ny=6200, steps_per_launch=3) == -6
    assert status_of(lbm, nx=6200, ny=6200, steps_per_launch=0) == 0    # two, on two descriptors


@pytest.mark.parametrize("spl", [3, 4, 8])
def test_a_batch_has_no_tile_form(lbm, spl):
    from paper_1308_2071_amd import _abi
    p = (_abi.LbmParams * 2)(lbm.make_params(nx=32, ny=32, steps_per_launch=spl),
                             lbm.make_params(nx=32, ny=32))
    n = C.c_size_t()
    assert _abi.library().lbm_batch_workspace_size(2, p, C.byref(n)) == -6   # UNSUPPORTED


def test_two_steps_per_launch_need_each_half_of_the_state_below_2_gib(lbm):
    """The two-step kernel addresses a state through buffer descriptors (one for a state below
    2^31 bytes, else two: planes 0-6 and 7-13) and drops the stores of lanes that own no node
    through an offset of 2^31, so each descriptor must cover less than 2^31 bytes."""
    # FP64: 4400^2 is 2.17 GB (two descriptors of 1.08 GB); 6100^2 has 7 planes of 2.10 GB in
    # all, 6200^2 of 2.16 GB
    assert status_of(lbm, nx=3500, ny=3500, dtype=1, steps_per_launch=2) == 0
    assert status_of(lbm, nx=4400, ny=4400, dtype=1, steps_per_launch=2) == 0
    assert status_of(lbm, nx=6100, ny=6100, dtype=1, steps_per_launch=2) == 0
    assert status_of(lbm, nx=6200, ny=6200, dtype=1, steps_per_launch=2) == -6  # UNSUPPORTED
    assert status_of(lbm, nx=6200, ny=6200, dtype=1, steps_per_launch=0) == 0   # single steps
    # FP32: 8700^2 has 7 planes of 2.12 GB, 8800^2 of 2.18 GB
    assert status_of(lbm, nx=8700, ny=8700, steps_per_launch=2) == 0
    assert status_of(lbm, nx=8800, ny=8800, steps_per_launch=2) == -6
    # the batched two-step kernel takes one descriptor per cavity: below 2 GiB each
    from paper_1308_2071_amd import _abi
    big = lbm.make_params(nx=6500, ny=6500, steps_per_launch=0)
    small = lbm.make_params(nx=64, ny=64, steps_per_launch=2)
    p = (_abi.LbmParams * 2)(small, big)
    n = C.c_size_t()
    assert _abi.library().lbm_batch_workspace_size(2, p, C.byref(n)) == -6
    p = (_abi.LbmParams * 2)(lbm.make_params(nx=64, ny=64), big)
    assert _abi.library().lbm_batch_workspace_size(2, p, C.byref(n)) == 0
