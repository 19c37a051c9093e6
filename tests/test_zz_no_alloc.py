"""lbm_run_noalloc, the entry point that allocates nothing: its results equal those of
lbm_init + lbm_step + lbm_observables (the existing entry points, same kernels) bitwise, on
consecutive calls that share the library's one device array, the second call with a smaller
cavity; a cavity beyond the array's 64 MiB is refused before any device work."""
import numpy as np
import pytest
import torch

from paper_1308_2071_amd import (Cavity, LbmError, lbm_run_noalloc, lbm_workspace_size,
                                 make_params, workloads)

pytestmark = pytest.mark.gpu

FIELDS = ("ux", "uy", "p", "T")
OBS = ("nu_hot", "nu_cold", "max_speed", "mass_err", "step", "diverged", "why", "T_min",
       "T_max", "phip_dev")


def reference(params, phi, K, phi_u, steps):
    cav = Cavity(params, phi=phi, K=K, phi_uniform=phi_u, device="cuda")
    cav.step(steps)
    o = cav.observables()
    cav.close()
    return o


def noalloc(params, phi, K, phi_u, steps):
    p = make_params(**params)
    dt = torch.float64 if params.get("dtype") == "fp64" else torch.float32
    cv = lambda t: None if t is None else t.to("cuda", dt).contiguous()
    out = {k: torch.full((p.ny, p.nx), float("nan"), dtype=dt, device="cuda") for k in FIELDS}
    s, o = lbm_run_noalloc(p, cv(phi), cv(K), phi_u, steps, out["ux"], out["uy"], out["p"],
                           out["T"])
    out.update({k: getattr(o, k) for k in OBS})
    out["status"] = s
    return out


def assert_same(a, b, what):
    for k in FIELDS:
        assert torch.equal(a[k], b[k]), (what, k)
    for k in ("nu_hot", "nu_cold", "max_speed", "mass_err", "T_min", "T_max", "phip_dev"):
        assert a[k] == b[k] or (np.isnan(a[k]) and np.isnan(b[k])), (what, k, a[k], b[k])
    assert a["step"] == b["step"] and bool(a["diverged"]) == bool(b["diverged"]), what
    assert a["status"] == b["status"] == 0, what


CASES = [
    # per-node medium, FP64, mixed walls; then a smaller uniform FP32 cavity, odd step count;
    # then two and three steps per launch forced on mid-size FP32 cavities (65 steps: 21 launches
    # of three and two single steps)
    ("per_node_fp64", dict(nx=300, ny=200, Ra=1e5, Pr=0.71, dtype="fp64",
                           bc=(1, 0, 0, 1), T_wall=(0.0, 0.2, 1.0, 0.0)), True, 0.6, 500),
    ("uniform_fp32", dict(nx=64, ny=48, Ra=1e4, Pr=1.0, Da=1e-2, dtype="fp32"), False, 0.45,
     301),
    ("fused_fp32", dict(nx=600, ny=400, Ra=1e6, Pr=0.71, dtype="fp32", steps_per_launch=2),
     True, 0.6, 64),
    ("fused3_fp32", dict(nx=500, ny=300, Ra=1e6, Pr=0.71, dtype="fp32", steps_per_launch=3,
                         bc=(0, 0, 1, 0), T_wall=(1.0, 0.0, 0.0, 0.4)), True, 0.6, 65),
]


def test_noalloc_equals_the_workspace_entry_points_on_consecutive_calls():
    sizes = []
    for name, params, per_node, phi_u, steps in CASES:
        phi = K = None
        if per_node:
            phi, K = (torch.from_numpy(a) for a in
                      workloads.random_medium(params["ny"], params["nx"], seed=params["nx"]))
        want = reference(params, phi, K, phi_u, steps)
        got = noalloc(params, phi, K, phi_u, steps)
        assert_same(got, want, name)
        sizes.append(lbm_workspace_size(make_params(**params)))
    assert sizes[1] < sizes[0]   # the second call is the smaller cavity


def test_noalloc_repeats_bitwise_after_a_larger_call():
    """The array keeps the last call's contents; a call must not depend on them."""
    small = CASES[1]
    a = noalloc(small[1], None, None, small[3], small[4])
    big = CASES[0]
    phi, K = (torch.from_numpy(x) for x in workloads.random_medium(200, 300, seed=300))
    noalloc(big[1], phi, K, big[3], 50)
    b = noalloc(small[1], None, None, small[3], small[4])
    assert_same(a, b, "repeat")


def test_noalloc_refuses_a_cavity_beyond_its_array():
    params = dict(nx=1500, ny=1500, Ra=1e6, Pr=0.71, dtype="fp32")
    assert lbm_workspace_size(make_params(**params)) > 64 << 20
    with pytest.raises(LbmError, match="LBM_E_NOMEM.*at most 67108864"):
        noalloc(params, None, None, 0.6, 10)
    with pytest.raises(LbmError, match="LBM_E_UNSUPPORTED"):
        noalloc(dict(nx=32, ny=32, checkpoint_every=10), None, None, 0.6, 10)
