"""Differentiable test-particle tracking on the GPU (pic_track_*) against the
FP64 oracle: the forward trajectories, and the adjoint gradient against the
oracle's complex-step derivatives, which share no arithmetic with the hand-
written adjoint.

* FP64: trajectories to 1e-10 and gradients to 1e-8 of their scale.
* FP32 (trajectory and adjoint in float32, sums in float64): final states
  within 3x of the oracle run with float32 state storage; gradients to 1e-3
  relative, the tolerance the polarization itself is held to.
* The checkpoint interval changes nothing (bit for bit).
* The torch autograd wrapper gives the adjoint's gradient, which also matches
  central differences of the GPU forward itself.
* c4 at full size (2^20 protons, 4000 steps, states every 100): sampled
  particles against tests/golden/c4_oracle.json (written by
  tests/golden/make_c4_golden.py, which calls only the oracle).
"""

import json
import os
import warnings

import numpy as np
import pytest

import oracle
import synth
from paper_2002_02211_amd import spinpic as S

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_oracle.json")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _small(seed=44, n=64, nsteps=300):
    spec = synth.tracking_preset("track_small", seed=seed, n=n, nsteps=nsteps)
    x, u, s = synth.make_beam(spec)
    rng = np.random.default_rng(seed + 1)
    u[:, :2] = rng.normal(0.0, 0.3, (n, 2))          # some transverse momentum
    s = s + rng.normal(0.0, 0.2, s.shape)             # spins off axis
    s /= np.linalg.norm(s, axis=1)[:, None]
    return spec, x, u, s


def _oracle_grads(spec, x, u, s, c):
    warnings.simplefilter("ignore")
    sp = spec["species"]
    args = (spec["E0"], spec["kp"], spec["dt"], spec["nsteps"], sp["Z"], sp["mu"], sp["a"])
    fin = oracle.tracking_forward(x, u, s, *args)
    d = oracle.per_particle_complex_step(x, u, s, *args, c)
    return fin, d


def _tracker(spec, precision, checkpoint=None):
    sp = spec["species"]
    return S.Tracker(spec["n"], Z=sp["Z"], mu=sp["mu"], a=sp["a"], dt=spec["dt"], nsteps=spec["nsteps"],
                     checkpoint=checkpoint or spec["checkpoint"], precision=precision)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


C = np.array([0.2, -0.3, 1.0])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_beam_forward_and_gradient(precision):
    spec, x, u, s = _small()
    _say("track_small", precision)
    (xf, uf, sf), (dE0, dkp, dx, du, ds) = _oracle_grads(spec, x, u, s, C)
    n = spec["n"]
    tr = _tracker(spec, precision)
    P, gx_f, gu_f, gs_f = tr.forward(spec["E0"], spec["kp"], x, u, s, want_state=True)
    gth, gx, gu, gs, each = tr.backward(C, per_particle_theta=True)
    tr.close()
    errs = {"x": _rel(gx_f, xf), "u": _rel(gu_f, uf), "s": float(np.max(np.abs(gs_f - sf))),
            "P": float(np.max(np.abs(P - sf.mean(axis=0)))),
            "dE0": abs(gth[0] - dE0.mean()) / abs(dE0.mean()), "dkp": abs(gth[1] - dkp.mean()) / abs(dkp.mean()),
            "dx0": _rel(gx, dx / n), "du0": _rel(gu, du / n), "ds0": _rel(gs, ds / n),
            "each": max(_rel(each[:, 0], dE0 / n), _rel(each[:, 1], dkp / n))}
    _say(precision, " ".join("%s %.2e" % kv for kv in errs.items()))
    if precision == "fp64":
        assert errs["x"] < 1e-10 and errs["u"] < 1e-10 and errs["s"] < 1e-10 and errs["P"] < 1e-12
        for k in ("dE0", "dkp", "dx0", "du0", "ds0", "each"):
            assert errs[k] < 1e-8, (k, errs[k])
    else:
        # states: within 3x of the exact method with float32 storage (small
        # momentum kicks added to u_z ~ 20, whose float32 ulp is 2e-6, cost
        # that much by themselves); gradients: 1e-3 relative, the tolerance
        # the polarization itself is held to
        sp = spec["species"]
        x32, u32, s32 = oracle.tracking_forward(x, u, s, spec["E0"], spec["kp"], spec["dt"], spec["nsteps"],
                                                sp["Z"], sp["mu"], sp["a"], store_fp32=True)
        ref = {"x": _rel(x32, xf), "u": _rel(u32, uf), "s": float(np.max(np.abs(s32 - sf)))}
        _say("float32 storage alone:", " ".join("%s %.2e" % kv for kv in ref.items()))
        for k in ("x", "u", "s"):
            assert errs[k] <= 3.0 * ref[k] + 1e-7, (k, errs[k], ref[k])
        assert errs["P"] < 1e-6
        for k in ("dE0", "dkp", "dx0", "du0", "ds0", "each"):
            assert errs[k] < 1e-3, (k, errs[k])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_checkpoint_interval_changes_nothing(precision):
    spec, x, u, s = _small(seed=7, n=40, nsteps=120)
    _say("checkpoint invariance", precision)
    ref = None
    for K in (1, 7, 40, 120, 500):
        tr = _tracker(spec, precision, checkpoint=K)
        P = tr.forward(spec["E0"], spec["kp"], x, u, s)
        out = (P,) + tuple(tr.backward(C, per_particle_theta=True))
        tr.close()
        if ref is None:
            ref = out
            continue
        for a, b in zip(out, ref):
            np.testing.assert_array_equal(a, b)


def test_edge_cases():
    spec, x, u, s = _small(seed=9, n=5, nsteps=0)
    tr = _tracker(spec, "fp64", checkpoint=10)
    with pytest.raises(S.PicError) as e:
        tr.backward(C)
    assert e.value.code == S.PIC_ESTATE
    P = tr.forward(0.1, 0.1, x, u, s)
    np.testing.assert_allclose(P, s.mean(axis=0), rtol=0, atol=1e-15)
    gth, gx, gu, gs = tr.backward(C)
    assert np.all(gth == 0) and np.all(gx == 0) and np.all(gu == 0)
    np.testing.assert_allclose(gs, np.tile(C / 5, (5, 1)), rtol=1e-15)
    bad = x.copy()
    bad[2, 1] = np.nan
    with pytest.raises(S.PicError) as e:
        tr.forward(0.1, 0.1, bad, u, s)
    assert e.value.code == S.PIC_EINVAL
    tr.close()
    # one particle
    spec, x, u, s = _small(seed=10, n=1, nsteps=50)
    (xf, uf, sf), (dE0, dkp, dx, du, ds) = _oracle_grads(spec, x, u, s, C)
    tr = _tracker(spec, "fp64", checkpoint=16)
    P = tr.forward(spec["E0"], spec["kp"], x, u, s)
    gth, gx, gu, gs = tr.backward(C)
    tr.close()
    assert np.max(np.abs(P - sf[0])) < 1e-12
    assert abs(gth[0] - dE0[0]) <= 1e-9 * abs(dE0[0]) and _rel(gu, du) < 1e-8


def test_torch_autograd_gives_the_adjoint_and_matches_differences():
    import torch
    spec, x, u, s = _small(seed=12, n=32, nsteps=200)
    _say("torch autograd")
    tr = _tracker(spec, "fp64", checkpoint=25)
    E0 = torch.tensor(spec["E0"], dtype=torch.float64, requires_grad=True)
    kp = torch.tensor(spec["kp"], dtype=torch.float64, requires_grad=True)
    xt = torch.tensor(x, requires_grad=True)
    ut = torch.tensor(u, requires_grad=True)
    st = torch.tensor(s, requires_grad=True)
    P = S.wake_polarization(tr, E0, kp, xt, ut, st)
    w = torch.tensor(C)
    # an unrelated forward in between: the backward recomputes its own run
    tr.forward(0.3, 0.2, x, u, s)
    (w @ P).backward()
    tr.forward(spec["E0"], spec["kp"], x, u, s)
    gth, gx, gu, gs = tr.backward(C)
    assert E0.grad.item() == gth[0] and kp.grad.item() == gth[1]
    np.testing.assert_array_equal(ut.grad.numpy(), gu)
    np.testing.assert_array_equal(xt.grad.numpy(), gx)

    def J(e0, k):
        return float(C @ tr.forward(e0, k, x, u, s))

    for i, (base, h) in enumerate(((spec["E0"], 1e-3), (spec["kp"], 1e-4))):
        f = (lambda d: J(base + d, spec["kp"])) if i == 0 else (lambda d: J(spec["E0"], base + d))
        fd = (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)
        assert abs(gth[i] - fd) <= 1e-6 * abs(fd), (i, gth[i], fd)
    tr.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_c4_full_size_sampled(precision):
    with open(GOLDEN) as f:
        gold = json.load(f)
    spec = synth.tracking_preset("c4")
    _say("c4 full size", precision)
    x, u, s = synth.make_beam(spec)
    tr = _tracker(spec, precision)
    P, xf, uf, sf = tr.forward(spec["E0"], spec["kp"], x, u, s, want_state=True)
    gth, gx, gu, gs, each = tr.backward(gold["c"], per_particle_theta=True)
    t = tr.timing()
    tr.close()
    n = spec["n"]
    idx = np.array(gold["index"])
    np.testing.assert_allclose(P, sf.mean(axis=0), rtol=0, atol=1e-12)
    assert abs(gth[0] - each[:, 0].sum()) <= 1e-12 * abs(gth[0]) + 1e-300
    errs = {"x": _rel(xf[idx], np.array(gold["x"])), "u": _rel(uf[idx], np.array(gold["u"])),
            "s": float(np.max(np.abs(sf[idx] - np.array(gold["s"])))),
            "dE0": _rel(each[idx, 0], np.array(gold["d_dE0"]) / n),
            "dkp": _rel(each[idx, 1], np.array(gold["d_dkp"]) / n),
            "dx0": _rel(gx[idx], np.array(gold["d_dx0"]) / n),
            "du0": _rel(gu[idx], np.array(gold["d_du0"]) / n),
            "ds0": _rel(gs[idx], np.array(gold["d_ds0"]) / n)}
    _say(precision, "forward %.1f ms backward %.1f ms" % (t["forward_ms"], t["backward_ms"]),
         " ".join("%s %.2e" % kv for kv in errs.items()))
    if precision == "fp64":
        for k, v in errs.items():
            assert v < (1e-9 if k in ("x", "u", "s") else 1e-7), (k, v)
    else:
        ref32 = gold["store_fp32"]
        ref = {"x": _rel(np.array(ref32["x"]), np.array(gold["x"])),
               "u": _rel(np.array(ref32["u"]), np.array(gold["u"])),
               "s": float(np.max(np.abs(np.array(ref32["s"]) - np.array(gold["s"]))))}
        _say("float32 storage alone:", " ".join("%s %.2e" % kv for kv in ref.items()))
        for k in ("x", "u", "s"):
            assert errs[k] <= 3.0 * ref[k] + 1e-7, (k, errs[k], ref[k])
        for k in ("dE0", "dkp", "dx0", "du0", "ds0"):
            assert errs[k] < 1e-3, (k, errs[k])
