"""The FFT-path autotuner through the C ABI: every candidate it tries must
reproduce the default launch (none rejected), its choices must leave complete
and correct outputs, and later launches with the tuned plan must still match
the CPU FP64 oracle to the float bound (1e-5 relative RMS per fluid and
component)."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_10812_amd import torch_ops
    return torch_ops


@pytest.fixture(scope="module")
def W():
    from paper_2506_10812_amd import workloads
    return workloads


def rel_rms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle_check(F, i, w, tol=1e-5):
    nr, nphi, nf = w["n_r"], w["n_phi"], len(w["h"])
    sig32 = torch.tensor(w["sigma"], dtype=torch.float32).double().numpy()
    rr, rp = O.field_table(nr, nphi, w["r_min"], w["r_max"], w["h"], sig32)
    gr = F.g_r[i].double().cpu().numpy().reshape(nf, -1)
    gp = F.g_phi[i].double().cpu().numpy().reshape(nf, -1)
    for b in range(nf):
        assert rel_rms(gr[b], rr[b]) < tol, (i, b, rel_rms(gr[b], rr[b]))
        assert rel_rms(gp[b], rp[b]) < tol, (i, b, rel_rms(gp[b], rp[b]))


def test_tuner_mixed_batch(T, W, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SG_TUNE_CACHE", str(cache))
    # lengths with and without a small radix (16, 32, 128, 256, 1024 / 64, 512)
    specs = [W.bifluid_fft(seed=41, n_r=64, n_phi=128), W.single_fft(seed=42, n_r=128, n_phi=256),
             W.single_fft(seed=43, n_r=32, n_phi=512), W.bifluid_fft(seed=44, n_r=16, n_phi=64),
             W.single_fft(seed=45, n_r=8, n_phi=32), W.bifluid_fft(seed=46, n_r=256, n_phi=16)]
    print("tuner: mixed batch of", len(specs), "discs", flush=True)
    F = T.FFTField(specs)
    for i, s in enumerate(specs):
        F.set_sigma(i, s["sigma"])
    F.run()
    torch.cuda.synchronize()
    ref = [(F.g_r[i].clone(), F.g_phi[i].clone()) for i in range(len(specs))]
    for i in range(len(specs)):
        F.g_r[i].zero_()
        F.g_phi[i].zero_()
    res = F.tune()
    torch.cuda.synchronize()
    classes = set()
    for p in (1, 2, 3):
        for s in specs:
            classes.add((p, 2 * s["n_r"] if p == 2 else s["n_phi"], len(s["h"])))
    assert len(res) == len(classes)
    assert {(r["pass"], r["length"], r["n_fluids"]) for r in res} == classes
    for r in res:
        print("  ", r, flush=True)
        assert r["rejected"] == 0, r
        assert r["candidates"] >= 3, r
        assert r["cluster"] in (1, 2, 4, 8) and r["small_radix_first"] in (0, 1), r
        assert r["ms_best"] <= r["ms_default"] * 1.0001, r
        assert r["rel_best"] <= 1e-5, r
    # the tuning call leaves complete outputs (another radix order rounds
    # differently: same float bound as against the oracle)
    for i in range(len(specs)):
        for got, want in zip((F.g_r[i], F.g_phi[i]), ref[i]):
            g, w = got.double().cpu().numpy(), want.double().cpu().numpy()
            print(f"  disc {i} tuned vs default rel-RMS {rel_rms(g, w):.2e}", flush=True)
            assert rel_rms(g, w) < 1e-5, (i, rel_rms(g, w))
    # the tuned plan: fresh launches, checked against the oracle
    for i in range(len(specs)):
        F.g_r[i].zero_()
        F.g_phi[i].zero_()
    F.run()
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        _oracle_check(F, i, s)
    lines = cache.read_text().split("\n")
    assert len([ln for ln in lines if ln.strip()]) >= len(classes)


def test_tuner_three_and_four_groups(T, W):
    """Launch classes with three and four groups (their column pass holds one
    source's spectra at a time): every candidate reproduces the reference and
    the tuned plan matches the oracle."""
    rng = np.random.default_rng(31)
    specs = []
    for nf, nr, nphi in ((3, 32, 64), (4, 64, 32)):
        base = W.bifluid_fft(seed=nr + nf, n_r=nr, n_phi=nphi)
        sig = np.concatenate([base["sigma"], base["sigma"][1:2] * rng.uniform(0.5, 2.0, (nf - 2, nr, nphi))])
        specs.append(dict(base, h=[0.05, 0.005, 0.02, 0.01][:nf], sigma=sig))
    print("tuner: three- and four-group discs", flush=True)
    F = T.FFTField(specs)
    for i, s in enumerate(specs):
        F.set_sigma(i, s["sigma"])
    res = F.tune()
    torch.cuda.synchronize()
    for r in res:
        print("  ", r, flush=True)
        assert r["rejected"] == 0 and r["rel_best"] <= 1e-5, r
    for i in range(len(specs)):
        F.g_r[i].zero_()
        F.g_phi[i].zero_()
    F.run()
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        _oracle_check(F, i, s)
