"""GPU checks of the precision form against the FP64 oracle at the 1352x760,
128-label, 6-level, 12-half-sweep workload, and of the autotuner's table."""
import json

import numpy as np
import pytest
import torch

import oracle
from synth import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("pset", ["int", "real"])
def test_precision_form_vs_fp64(dev, pset):
    """FP32 / FP16 / BF16 message storage against the FP64 oracle.  Integer
    parameter set: every message is an integer <= lambda*tau = 20, exact in
    all three formats, so labels and messages must match bit for bit.
    Real-valued set: at most 0.5% of pixels more than one label off, FP32
    messages within 1e-4 * lambda * tau but for a few near-tie entries, 16-bit
    messages within their format's rounding of FP64 and equal to the oracle
    that emulates the 16-bit storage, but for near-tie entries."""
    import paper_1902_09733_amd as bp
    wl = workload("aerial1352x760_L128")
    L, levels, K = wl["num_labels"], wl["levels"], wl["iters"]
    rgb_mode, lam, tau = (0, 10.0, 2.0) if pset == "int" else (1, 7.3, 2.6)
    left = torch.from_numpy(wl["left"]).to(dev)
    right = torch.from_numpy(wl["right"]).to(dev)
    cost = bp.cost_volume(left, right, L, 20.0, rgb_mode=rgb_mode)
    o = oracle.run(cost.double().cpu().numpy(), levels, K, lam, tau, want_msgs=True)
    report, r_msgs, d_of = {}, {}, {}
    for fmt in ("f32", "f16", "bf16"):
        r = bp.run(cost, bp.BPParams(levels=levels, iters=K, lam=lam, tau=tau, msg_dtype=fmt), want_msgs=True)
        torch.cuda.synchronize()
        d = r["disp"].cpu().numpy()
        r_msgs[fmt] = r["msgs"].double().cpu().numpy()
        d_of[fmt] = d
        diff = np.abs(r_msgs[fmt] - o["msgs"]) / (lam * tau)
        err = float(diff.max())
        bad = float((np.abs(d - o["disp"]) > 1).mean())
        report[fmt] = {"bad_pixel_vs_fp64": bad, "max_msg_err_over_lambda_tau": err,
                       "p99_9_msg_err_over_lambda_tau": float(np.quantile(diff, 0.999)),
                       "msg_entries_over_1e-4_lambda_tau": float((diff > 1e-4).mean()),
                       "msg_entries_over_1e-2_lambda_tau": float((diff > 1e-2).mean())}
        del diff
        del r
        if pset == "int":
            assert bad == 0.0 and err == 0.0, (fmt, report[fmt])
        else:
            assert bad <= 0.005, (fmt, report[fmt])
            rep = report[fmt]
            if fmt == "f32":
                # The 1e-4 * lambda * tau message bar holds for every entry
                # but a few near-tie senders, whose two near-equal minimisers
                # FP32 and FP64 order differently (measured: 2.5e-6 of the
                # entries, the largest 0.017 lambda * tau; 99.9% within 2e-7).
                assert rep["msg_entries_over_1e-4_lambda_tau"] <= 1e-5, (fmt, rep)
                assert rep["p99_9_msg_err_over_lambda_tau"] <= 1e-4, (fmt, rep)
            else:
                # 16-bit rows: the format's rounding (99.9% within 2.3e-4 /
                # 1.3e-3 lambda * tau for FP16 / BF16), full-range changes
                # only at near-tie senders.
                assert rep["p99_9_msg_err_over_lambda_tau"] <= 4e-3, (fmt, rep)
                assert rep["msg_entries_over_1e-2_lambda_tau"] <= 1e-3, (fmt, rep)
                # Against the oracle that rounds every stored message the same
                # way (its arithmetic FP64, the GPU's FP32): identical but for
                # near-tie entries (measured: 99.9% equal, 2.3e-6 / 7.9e-6 of
                # the entries beyond 8 of the format's ulps at lambda * tau,
                # labels off by more than one at 1e-6 / 6.7e-5 of the pixels).
                mode = oracle.STORE_F16 if fmt == "f16" else oracle.STORE_BF16
                o16 = oracle.run(cost.double().cpu().numpy(), levels, K, lam, tau, want_msgs=True, store_mode=mode)
                ulp = 2.0 ** -10 if fmt == "f16" else 2.0 ** -7
                d16 = np.abs(r_msgs[fmt] - o16["msgs"]) / (ulp * lam * tau)
                rep["vs_store_oracle_max_ulps"] = float(d16.max())
                rep["vs_store_oracle_p99_9_ulps"] = float(np.quantile(d16, 0.999))
                rep["vs_store_oracle_entries_over_8_ulps"] = float((d16 > 8).mean())
                rep["vs_store_oracle_labels_off_by_more_than_1"] = float((np.abs(d_of[fmt] - o16["disp"]) > 1).mean())
                del d16, o16
                assert rep["vs_store_oracle_p99_9_ulps"] <= 1.0, (fmt, rep)
                assert rep["vs_store_oracle_entries_over_8_ulps"] <= 1e-4, (fmt, rep)
                assert rep["vs_store_oracle_labels_off_by_more_than_1"] <= 1e-3, (fmt, rep)
        r_msgs.pop(fmt)
    print("precision", pset, json.dumps(report))


def test_tune_table_is_used_and_exact(dev, tmp_path):
    """The autotuner's table changes launch shapes only: runs that read a
    table (here forcing each candidate in turn) equal the oracle bit for bit."""
    import paper_1902_09733_amd as bp
    from paper_1902_09733_amd import _abi, tune
    best, results = tune.tune_shape(96, 64, 64, "f32", 3, 6, dev)
    assert best is not None and len(results) >= 2
    rng = np.random.default_rng(1)
    cost = rng.integers(0, 21, size=(64, 64, 96)).astype(np.float32)
    o = oracle.run(cost.astype(np.float64), 3, 6, 10.0, 2.0, want_msgs=True)
    c = torch.from_numpy(cost).to(dev)
    table = tmp_path / "table.txt"
    try:
        for pm_from, variant, _ in results:
            table.write_text(f"# width height labels fmt levels pm_from variant us\n96 64 64 0 3 {pm_from} {variant} 1.0\n")
            assert _abi.lib().bp_load_tune_table(str(table).encode()) == 0
            r = bp.run(c, bp.BPParams(levels=3, iters=6, lam=10.0, tau=2.0), want_msgs=True)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(r["disp"].cpu().numpy(), o["disp"])
            np.testing.assert_array_equal(r["msgs"].cpu().numpy().astype(np.float64), o["msgs"])
    finally:
        _abi.lib().bp_load_tune_table(None)
