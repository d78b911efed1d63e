"""The indirect term (SG_INDIRECT) through the C ABI against the CPU FP64
oracle: FFT path (float, 1e-5 relative RMS per fluid and component, and the
indirect part alone to 1e-5), direct path in double (1e-12 of max |g|) and in
float, general per-cell H, and the FFT-path adjoint with the term."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_10812_amd as m
    return m


@pytest.fixture(scope="module")
def T(sg):
    from paper_2506_10812_amd import torch_ops
    return torch_ops


@pytest.fixture(scope="module")
def W():
    from paper_2506_10812_amd import workloads
    return workloads


def rel_rms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _lopsided(w, seed):
    """The workload's Sigma times an m = 1 lopsidedness, so that the disc pulls
    the star (an axisymmetric disc has no indirect term)."""
    rng = np.random.default_rng(seed)
    nphi = w["n_phi"]
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    w = dict(w)
    w["sigma"] = w["sigma"] * (1 + 0.3 * np.cos(phi - rng.uniform(0, 2 * np.pi)))[None, None, :]
    return w


@pytest.mark.parametrize("nr,nphi,nf", [(16, 32, 1), (32, 64, 2), (64, 128, 2), (4, 8, 2)])
def test_fft_path_indirect_full_field(sg, T, nr, nphi, nf, W):
    print(f"indirect term, fft path {nr}x{nphi} nf={nf}", flush=True)
    base = W.bifluid_fft(seed=nr + 7, n_r=nr, n_phi=nphi) if nf == 2 else \
        W.single_fft(seed=nr + 7, n_r=nr, n_phi=nphi)
    w = _lopsided(base, nr)
    F0 = T.FFTField([w])
    F1 = T.FFTField([w], flags=sg.INDIRECT)
    for F in (F0, F1):
        F.set_sigma(0, w["sigma"])
        F.run()
    torch.cuda.synchronize()
    sig32 = torch.tensor(w["sigma"], dtype=torch.float32).double().numpy()
    rr, rp = O.field_table(nr, nphi, w["r_min"], w["r_max"], w["h"], sig32)
    AB = O.indirect(nr, nphi, w["r_min"], w["r_max"], w["h"], sig32)
    ir, ip = O.indirect_field(nr, nphi, AB)
    gr = F1.g_r[0].double().cpu().numpy().reshape(nf, -1)
    gp = F1.g_phi[0].double().cpu().numpy().reshape(nf, -1)
    dr = gr - F0.g_r[0].double().cpu().numpy().reshape(nf, -1)
    dp = gp - F0.g_phi[0].double().cpu().numpy().reshape(nf, -1)
    scale = max(np.abs(rr).max(), np.abs(rp).max())
    for b in range(nf):
        assert rel_rms(gr[b], rr[b] + ir) < 1e-5, (b, rel_rms(gr[b], rr[b] + ir))
        assert rel_rms(gp[b], rp[b] + ip) < 1e-5, (b, rel_rms(gp[b], rp[b] + ip))
        # the indirect part alone (float rounding of g bounds it)
        assert np.abs(dr[b] - ir).max() < 1e-5 * scale + 1e-5 * np.abs(ir).max()
        assert np.abs(dp[b] - ip).max() < 1e-5 * scale + 1e-5 * np.abs(ip).max()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_direct_indirect_general_H(sg, T, dtype):
    print(f"indirect term, direct path {dtype}, per-cell H", flush=True)
    nr, nphi, nf = 12, 20, 2
    rng = np.random.default_rng(17)
    rmin, rmax = 0.3, 3.0
    sig = rng.uniform(0.1, 1.0, (nf, nr, nphi))
    du = np.log(rmax / rmin) / nr
    r = np.exp(np.log(rmin) + (np.arange(nr) + 0.5) * du)
    H = (np.array([0.06, 0.02])[:, None, None] * r[None, :, None]) * rng.uniform(0.7, 1.3, (nf, nr, nphi))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    sig_t = torch.tensor(sig, dtype=tdt, device="cuda")
    H_t = torch.tensor(H, dtype=tdt, device="cuda")
    g = sg.grid(nr, nphi, rmin, rmax)
    gr, gp = T.direct(g, None, sig_t, H=H_t, flags=sg.INDIRECT)
    torch.cuda.synchronize()
    sig_in = sig_t.double().cpu().numpy()
    H_in = H_t.double().cpu().numpy()
    rr, rp = O.field_pairwise(nr, nphi, rmin, rmax, [0.0, 0.0], sig_in, H=H_in)
    AB = O.indirect(nr, nphi, rmin, rmax, [0.0, 0.0], sig_in, H=H_in)
    ir, ip = O.indirect_field(nr, nphi, AB)
    got_r = gr.double().cpu().numpy().reshape(nf, -1)
    got_p = gp.double().cpu().numpy().reshape(nf, -1)
    tol = 1e-12 if dtype == "f64" else 1e-5
    for b in range(nf):
        want_r, want_p = rr[b] + ir, rp[b] + ip
        scale = max(np.abs(want_r).max(), np.abs(want_p).max())
        err = max(np.abs(got_r[b] - want_r).max(), np.abs(got_p[b] - want_p).max()) / scale
        assert err < tol, (b, err)


def test_adjoint_with_indirect(sg, T, W):
    """FFT-path adjoint with SG_INDIRECT: the transpose identity
    <lam, g(Sigma)> = <dL/dSigma, Sigma> (the forward is pinned above),
    dL/dSigma at sampled cells against the oracle's L = <lam, g + g_ind>
    differenced in Sigma (exact: L is linear in Sigma), and dL/dh against
    central differences of that L in h (eps = 1e-4 h; 1e-4 relative)."""
    print("adjoint with the indirect term, fft path 32x64 nf=2", flush=True)
    w = _lopsided(W.adjoint(n_r=32, n_phi=64), 21)
    nr, nphi, rmin, rmax, h = w["n_r"], w["n_phi"], w["r_min"], w["r_max"], list(w["h"])
    F = T.FFTField([w], flags=sg.WITH_DH | sg.INDIRECT)
    F.set_sigma(0, w["sigma"])
    F.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(22)
    lr = rng.standard_normal((2, nr, nphi)).astype(np.float32)
    lp = rng.standard_normal((2, nr, nphi)).astype(np.float32)
    lr_t, lp_t = torch.tensor(lr).cuda(), torch.tensor(lp).cuda()
    ds = torch.empty_like(F.sigma[0])
    dh = torch.empty(2, dtype=torch.float64, device="cuda")
    ws = torch.empty(sg.field_adjoint_workspace_bytes(F.discs[0]), dtype=torch.uint8, device="cuda")
    sg.field_adjoint(F.discs[0], lr_t, lp_t, ds, dh, ws)
    torch.cuda.synchronize()
    lhs = float((lr_t.double() * F.g_r[0].double()).sum() + (lp_t.double() * F.g_phi[0].double()).sum())
    rhs = float((ds.double() * F.sigma[0].double()).sum())
    print(f"  <lam, g> {lhs:.8e}  <dL/dSigma, Sigma> {rhs:.8e}", flush=True)
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)
    sig = F.sigma[0].double().cpu().numpy()
    lr64, lp64 = lr.astype(np.float64).reshape(2, -1), lp.astype(np.float64).reshape(2, -1)

    def L(sigma, hh):
        gr, gp = O.field_table(nr, nphi, rmin, rmax, hh, sigma)
        ir, ip = O.indirect_field(nr, nphi, O.indirect(nr, nphi, rmin, rmax, hh, sigma))
        return float(np.sum(lr64 * (gr + ir[None, :])) + np.sum(lp64 * (gp + ip[None, :])))

    L0 = L(sig, h)
    dsn = ds.double().cpu().numpy()
    scale = np.abs(dsn).max()
    for a, k in [(0, 0), (1, 5), (0, 777), (1, nr * nphi - 1), (0, 1500), (1, 1234)]:
        sp = sig.copy()
        sp.reshape(2, -1)[a, k] += 1.0
        want = L(sp, h) - L0
        got = dsn.reshape(2, -1)[a, k]
        print(f"  dL/dSigma[{a}][{k}] {got:.6e} oracle {want:.6e}", flush=True)
        assert abs(got - want) < 1e-5 * scale, (a, k, got, want)
    # the autograd function with indirect=True runs the same adjoint
    sg_t = F.sigma[0].clone().requires_grad_(True)
    h_t = torch.tensor(h, dtype=torch.float64, requires_grad=True)
    gr_t, gp_t = T.SGField.apply(sg_t, h_t, nr, nphi, rmin, rmax, True)
    ((gr_t.double() * lr_t.double()).sum() + (gp_t.double() * lp_t.double()).sum()).backward()
    assert torch.equal(gr_t, F.g_r[0]) and torch.equal(gp_t, F.g_phi[0])
    assert torch.equal(sg_t.grad, ds)
    assert torch.allclose(h_t.grad, dh.cpu(), rtol=1e-12, atol=0)
    dhn = dh.cpu().numpy()
    for a in range(2):
        e = 1e-4 * h[a]
        hp_, hm_ = list(h), list(h)
        hp_[a] += e
        hm_[a] -= e
        want = (L(sig, hp_) - L(sig, hm_)) / (2 * e)
        print(f"  dL/dh[{a}] {dhn[a]:.8e} oracle {want:.8e}", flush=True)
        assert abs(dhn[a] - want) < 1e-4 * abs(want), (a, dhn[a], want)
