"""Adjoint form: gradient of a macroscopic stress-strain curve with respect to
(tau0, K, y_c, c_gnd) through rve_adjoint_increment with checkpointed increments (GPU only).

Workload: the adjoint workload (100 grains, Cu, c_gnd = 1) on an 8^3 grid, first 6 increments
of its load path, FP64 at |dF| <= 1e-13.  The loss is the curve loss
L = sum_k (<P>_11,k - target_k)^2 against the synthetic target of
tests/golden/adjoint_cu64g100_8cubed.json (the oracle's curve at perturbed parameters plus
seeded noise)."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_cu64g100_8cubed.json")
OPTS = dict(newton_tol=1e-13, cg_tol=1e-12, max_cg=20000, max_newton=80)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_01946_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _curve(lib, rve, path, theta):
    import dataclasses
    r = dataclasses.replace(rve, material=synth.with_params(rve.material, theta))
    h = lib.Homogenizer([r], precision=lib.RVE_FP64, **OPTS)
    out = []
    for k in range(1, path.n_inc + 1):
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        out.append(h.macro()[0][0])
    h.close()
    return np.array(out)


def test_curve_loss_gradient_matches_central_differences_and_the_oracle(lib, golden):
    """dL/dtheta from the reverse pass (checkpoints every 2 increments, so that the replay of
    segments is exercised) against (a) central differences of the GPU forward, and (b) the
    oracle's own central-difference derivatives of the curve contracted with the same loss
    weights.  The forward solves stop at |dF| <= 1e-13, which leaves about 1e-13 of rounding
    noise on <P>: a relative step of 1e-6 moves the curve by 1e-6 of itself in tau0 but by only
    ~1e-9 in y_c, whose quotient then carries ~2e-4 of noise (measured), so the GPU quotient
    takes relative steps of 1e-5 (truncation error ~1e-9) and the 1e-6 quotient is printed
    beside it.  The reverse pass solves its multiplier to CG 1e-12.  Bar: 1e-4 relative per
    parameter (a wrong sign, a missing term of the chain or a transposed tangent give errors
    of order one)."""
    import torch
    from paper_1910_01946_amd.autograd import MacroCurve
    rve, path, theta = synth.adjoint_workload(n_override=golden["n"], n_inc_override=golden["n_inc"])
    target = torch.tensor(golden["target"], dtype=torch.float64)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    print("forward and reverse pass", flush=True)
    curve = MacroCurve.apply(th, rve, path, dict(precision=lib.RVE_FP64, **OPTS), 2)
    loss = torch.sum((curve - target) ** 2)
    loss.backward()
    grad = th.grad.numpy()
    c = curve.detach().numpy()
    w = 2.0 * (c - np.array(golden["target"]))
    print("curve", c, "oracle curve", golden["curve"], flush=True)
    assert np.max(np.abs(c - np.array(golden["curve"]))) <= 1e-10 * np.abs(c).max()
    # (b) the oracle's derivatives of the curve, contracted with the loss weights
    d_or = np.array(golden["dcurve_dtheta"]["1e-06"])
    d_or2 = np.array(golden["dcurve_dtheta"]["4e-06"])
    g_or = w @ d_or
    g_or_err = np.abs(w @ (d_or - d_or2))
    # (a) central differences of the GPU forward
    g_fd = np.zeros((2, 4))
    for j in range(4):
        for s_i, rel in enumerate((1e-5, 1e-6)):
            hstep = rel * theta[j]
            tp, tm = list(theta), list(theta)
            tp[j] += hstep
            tm[j] -= hstep
            print(f"central difference in {synth.ADJOINT_PARAMS[j]}, relative step {rel:g}", flush=True)
            Lp = np.sum((_curve(lib, rve, path, tp) - golden["target"]) ** 2)
            Lm = np.sum((_curve(lib, rve, path, tm) - golden["target"]) ** 2)
            g_fd[s_i, j] = (Lp - Lm) / (2 * hstep)
    for j, name in enumerate(synth.ADJOINT_PARAMS):
        e_fd = abs(grad[j] - g_fd[0, j]) / abs(g_fd[0, j])
        e_fd6 = abs(grad[j] - g_fd[1, j]) / abs(g_fd[1, j])
        e_or = abs(grad[j] - g_or[j]) / abs(g_or[j])
        print(f"{name}: reverse pass {grad[j]:.10e}, GPU differences {g_fd[0, j]:.10e} ({e_fd:.2e}; "
              f"step 1e-6: {e_fd6:.2e}), "
              f"oracle differences {g_or[j]:.10e} ({e_or:.2e}, the oracle's step error {g_or_err[j] / abs(g_or[j]):.1e})",
              flush=True)
        assert e_fd <= 1e-4
        assert e_or <= 1e-4 + 10 * g_or_err[j] / abs(g_or[j])


def test_per_increment_sensitivities_match_the_oracle(lib, golden):
    """d<P>_11,k / dtheta for the last and the first increment alone (unit weights), against
    the oracle's central-difference derivatives of the curve: the reverse pass of a single
    increment (no later increments) and the whole chain back to the initial state."""
    import torch
    from paper_1910_01946_amd.autograd import MacroCurve
    rve, path, theta = synth.adjoint_workload(n_override=golden["n"], n_inc_override=golden["n_inc"])
    d_or = np.array(golden["dcurve_dtheta"]["1e-06"])
    d_or2 = np.array(golden["dcurve_dtheta"]["4e-06"])
    for k in (golden["n_inc"], 1):
        th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
        curve = MacroCurve.apply(th, rve, path, dict(precision=lib.RVE_FP64, **OPTS), 5)
        curve[k - 1].backward()
        g = th.grad.numpy()
        for j, name in enumerate(synth.ADJOINT_PARAMS):
            ref = d_or[k - 1, j]
            step_err = abs(d_or[k - 1, j] - d_or2[k - 1, j])
            if abs(ref) < 1e-3 * np.abs(d_or[:, j]).max():
                # a parameter that has not reached this increment yet (K, y_c act through the
                # densities of later increments): both sides are (near) zero
                print(f"increment {k}, {name}: reverse pass {g[j]:.3e}, oracle {ref:.3e} (near zero)", flush=True)
                assert abs(g[j]) <= 1e-3 * np.abs(d_or[:, j]).max() + 10 * step_err
                continue
            e = abs(g[j] - ref) / abs(ref)
            print(f"increment {k}, {name}: reverse pass {g[j]:.10e}, oracle {ref:.10e} ({e:.2e})", flush=True)
            assert e <= 1e-4 + 10 * step_err / abs(ref)


def test_reverse_pass_refuses_an_rve_without_increments_and_bad_arguments(lib):
    import torch
    rve, path, theta = synth.adjoint_workload(n_override=8, n_inc_override=2)
    h = lib.Homogenizer([rve], precision=lib.RVE_FP64, **OPTS)
    Fpb = torch.zeros((9, rve.n_vox), dtype=torch.float64, device="cuda")
    rb = torch.zeros((12, rve.n_vox), dtype=torch.float64, device="cuda")
    tb = np.zeros(4)
    with pytest.raises(lib.RVEError) as e:
        h.adjoint_increment(path.mask, np.ones(9), Fpb, rb, tb)
    assert e.value.code == -5
    h.step(path.F_bar[1], path.mask, path.P_bar[1], path.dt)
    with pytest.raises(lib.RVEError) as e:
        h.adjoint_increment(path.mask, np.full(9, np.nan), Fpb, rb, tb)
    assert e.value.code == -1
    h.close()
