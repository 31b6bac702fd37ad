"""Learned compounding on the GPU: feature packing against its definition, linearity of the
compound in the transmits, and a short training run that beats the scaled few-angle sum."""

import types

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda"


def bf16_round(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).float().numpy()


def test_features_rescale_and_output_match_definition():
    from paper_2604_06257_amd import compound as C
    r = np.random.default_rng(3)
    A, V, cin, gain = 3, 1000, 8, 11 / 3
    ys = (r.standard_normal((A, V)) + 1j * r.standard_normal((A, V))).astype(np.complex64)
    ysd = torch.as_tensor(ys, device=DEV)
    x = torch.full((V, cin), 9.0, dtype=torch.bfloat16, device=DEV)
    base = torch.zeros((V, 2), dtype=torch.float32, device=DEV)
    scale = torch.zeros(2, dtype=torch.float32, device=DEV)
    work = torch.zeros(4, dtype=torch.float32, device=DEV)
    C.compound_features(ysd, gain, x, base, work, scale)
    s = ys.astype(np.complex128).sum(0)
    rms = np.sqrt(np.mean(np.abs(s) ** 2))
    sc = scale.cpu().numpy()
    assert sc[0] == pytest.approx(rms, rel=1e-5) and sc[1] == pytest.approx(1 / rms, rel=1e-5)
    xr = np.zeros((V, cin))
    xr[:, 0:2 * A:2] = (ys.real / sc[0]).T
    xr[:, 1:2 * A:2] = (ys.imag / sc[0]).T
    got = x.float().cpu().numpy()
    np.testing.assert_allclose(got, bf16_round(xr), rtol=1e-2, atol=1e-6)
    assert not got[:, 2 * A:].any()
    b = base.cpu().numpy()
    np.testing.assert_allclose(b[:, 0] + 1j * b[:, 1], gain * s / rms, rtol=1e-5, atol=1e-5)
    # rescale and output
    y = torch.as_tensor(s.astype(np.complex64), device=DEV)
    yn = torch.empty_like(y)
    C.compound_rescale(y, scale, yn)
    np.testing.assert_allclose(yn.cpu().numpy(), s / rms, rtol=1e-5, atol=1e-6)
    net = torch.as_tensor(r.standard_normal((V, 16)).astype(np.float32), device=DEV)
    out = torch.empty((V, 1), dtype=torch.complex64, device=DEV)
    C.compound_output(net, base, scale, out)
    n = net.cpu().numpy()
    ref = (b[:, 0] + n[:, 0] + 1j * (b[:, 1] + n[:, 1])) * rms
    np.testing.assert_allclose(out.cpu().numpy()[:, 0], ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())


def _small_task():
    from paper_2604_06257_amd import das
    from paper_2604_06257_amd.compound import LearnedCompounding
    from paper_2604_06257_amd.train_compound import geometry
    geo = geometry("small")
    p = geo["params"]
    elem = torch.as_tensor(geo["elem"].astype(np.float32), device=DEV)
    vox = torch.as_tensor(geo["vox"].astype(np.float32), device=DEV)
    tx = das.tx_plane_wave(vox, geo["angles"], p["c"])
    T, E, V = geo["angles"].shape[0], elem.shape[0], vox.shape[0]
    params = das.Params(T, E, p["n_samples"], 1, V, p["c"], p["fs"], p["fd"], p["t0"], p["f_number"],
                        p["tukey_alpha"])
    return geo, LearnedCompounding(params, elem, vox, tx, geo["dims"], geo["input_idx"])


def test_full_compound_is_the_sum_of_single_angle_volumes():
    """Delay-and-sum is linear in the transmits: the 11-angle plan equals the sum of 11 one-angle plans."""
    from paper_2604_06257_amd import das
    from synth import echo_iq_gpu
    geo, lc = _small_task()
    p = geo["params"]
    scat, amp = geo["phantom"](0)
    iq = echo_iq_gpu(geo["elem"], geo["angles"], scat, amp, n_samples=p["n_samples"], n_frames=1, c=p["c"],
                     fs=p["fs"], fc=p["fc"], fd=p["fd"], t0=p["t0"])
    full = lc.full_compound(iq).cpu().numpy()[:, 0].astype(np.complex128)
    one = das.Params(**{**lc.params.__dict__, "n_tx": 1})
    acc = np.zeros_like(full)
    vox = torch.as_tensor(geo["vox"].astype(np.float32), device=DEV)
    tx = das.tx_plane_wave(vox, geo["angles"], p["c"])
    elem = torch.as_tensor(geo["elem"].astype(np.float32), device=DEV)
    for t in range(lc.params.n_tx):
        with das.Plan(one, elem, vox, tx[t:t + 1].contiguous()) as plan:
            acc += plan.execute(iq[t:t + 1]).cpu().numpy()[:, 0]
    assert np.linalg.norm(full - acc) <= 1e-5 * np.linalg.norm(full)
    # the input-angle volumes (per-transmit output of one plan) are the one-angle plans' volumes
    assert lc.per_tx
    ys = lc.beamform_inputs(lc.input_iq(iq)).cpu().numpy()
    for a, t in enumerate(lc.input_idx):
        with das.Plan(one, elem, vox, tx[t:t + 1].contiguous()) as plan:
            y1 = plan.execute(iq[t:t + 1]).cpu().numpy()[:, 0]
            np.testing.assert_allclose(ys[a], y1, rtol=1e-5, atol=1e-6 * np.abs(y1).max())
    lc.close()


def test_learned_compounding_beats_scaled_input_sum():
    from paper_2604_06257_amd.train_compound import run
    args = types.SimpleNamespace(geometry="small", n_train=48, n_val=4, n_test=8, steps=600, lr=2e-3, seed=0,
                                 log_every=200, eval_every=200)
    res = run(args, log=print)
    print(res)
    nr = res["test_nrmse_db"]
    # held-out phantoms: the network must beat the scaled sum of the 3 input angles by >= 1 dB
    assert nr["network"] <= nr["scaled_input_sum"] - 1.0, nr
    assert res["speedup"] > 0


def test_c5_stored_weights_reproduce_the_learned_gain_on_held_out_phantoms():
    """The weights stored with the package (trained on 1800 c5 phantoms: 96^3 grid, 32 x 32 array, 11 plane waves)
    on 6 held-out phantoms generated here from the training run's test seeds: the network's NRMSE against the
    11-angle compound must beat (11/3) x the 3-angle sum by >= 2.5 dB (the full 100-phantom test set gave +3.17 dB),
    and the learned path must be faster than 11-angle DAS."""
    from paper_2604_06257_amd import train_compound
    import os
    path = os.path.join(os.path.dirname(train_compound.__file__), "weights", "unet_c5.npz")
    r = train_compound.evaluate_checkpoint(path, n_test=6)
    print(r)
    nr = r["nrmse_db_vs_full_compound"]
    assert nr["network"] <= nr["scaled_input_sum"] - 2.5, nr
    assert r["speedup"] > 1.5, r["ms"]
