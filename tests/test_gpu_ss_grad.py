"""dL/dH(r) on the semi-spectral path (sg_ss_grad_H) through the C ABI.

Checked against
  * central differences of the CPU FP64 oracle's L = <lam, g(H)> (pairwise
    sum with per-ring H broadcast to every cell, plus the oracle's indirect
    field where flagged), one ring and fluid at a time, on small log and
    uniform grids with flaring, a temperature gap, odd n_r, up to three
    groups, the own cell dropped or kept; likewise for the potential
    operators with L = <lam_r, Phi(H)>;
  * the oracle's dL/dh_f for H_f = h_f r: by the chain rule
    sum_i r_i dL/dH_f(r_i) = dL/dh_f (the offset-table derivative sum);
  * at the App. D size, a directional derivative of the GPU forward (itself
    pinned to the oracle), table rebuilt at H +- eps dH.
Bound: lam and Sigma enter as float32 half spectra (2^-24 relative each)
and the derivative operators are accumulated in double, so the gradient
carries a few float roundings per term (about 1e-7 of max |dL/dH| seen);
the bound is 1e-6 of max |dL/dH| per element and 1e-6 relative in L2."""
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


def say(msg):
    print(msg, flush=True)


def lams(shape, seed):
    g = np.random.default_rng(seed)
    return (g.standard_normal(shape).astype(np.float32), g.standard_normal(shape).astype(np.float32))


def gpu_grad(sg, T, w, flags, lr, lp):
    nf = w["sigma"].shape[0]
    S = T.SemiSpectral(w["n_r"], w["n_phi"], w["r_min"], w["r_max"], nf, flags)
    S.refresh(w["H"])
    S.sigma.copy_(torch.tensor(w["sigma"], dtype=torch.float32))
    H = torch.tensor(w["H"], dtype=torch.float64, device="cuda")
    dH = torch.empty_like(H)
    ws = torch.empty(sg.ss_grad_H_workspace_bytes(S.disc), dtype=torch.uint8, device="cuda")
    sg.ss_grad_H(S.disc, H, torch.tensor(lr).cuda(), torch.tensor(lp).cuda(), dH, ws)
    torch.cuda.synchronize()
    return S, dH.cpu().numpy()


def oracle_L(w, H, flags, lr, lp):
    nf, nr, nphi = w["sigma"].shape
    sig = w["sigma"].astype(np.float32).astype(np.float64)
    Hc = np.repeat(H[:, :, None], nphi, axis=2)
    of = (O.EXCLUDE_SELF if flags & 1 else 0) | (O.LINEAR_R if flags & 64 else 0)
    gr, gp = O.field_pairwise(nr, nphi, w["r_min"], w["r_max"], [0.0] * nf, sig, H=Hc, flags=of)
    lr = lr.reshape(nf, -1).astype(np.float64)
    lp = lp.reshape(nf, -1).astype(np.float64)
    L = float(np.sum(lr * gr) + np.sum(lp * gp))
    if flags & 4:
        AB = O.indirect(nr, nphi, w["r_min"], w["r_max"], [0.0] * nf, sig, H=Hc,
                        flags=O.LINEAR_R if flags & 64 else 0)
        ir, ip = O.indirect_field(nr, nphi, AB)
        L += float(np.sum(lr * ir[None, :]) + np.sum(lp * ip[None, :]))
    return L


def oracle_L_pot(w, H, flags, lr):
    """L = <lam_r, Phi(H)> with the oracle's pairwise potential (per-ring H at
    every cell); the potential operators write Phi to g_r."""
    nf, nr, nphi = w["sigma"].shape
    sig = w["sigma"].astype(np.float32).astype(np.float64)
    Hc = np.repeat(H[:, :, None], nphi, axis=2)
    of = (O.EXCLUDE_SELF if flags & 1 else 0) | (O.LINEAR_R if flags & 64 else 0)
    pot = O.potential_pairwise(nr, nphi, w["r_min"], w["r_max"], [0.0] * nf, sig, H=Hc, flags=of)
    return float(np.sum(lr.reshape(nf, -1).astype(np.float64) * pot))


def oracle_fd(w, flags, lr, lp, rel=1e-4):
    H0 = np.array(w["H"], dtype=np.float64)
    out = np.zeros_like(H0)
    for f in range(H0.shape[0]):
        for i in range(H0.shape[1]):
            e = rel * H0[f, i]
            Hp = H0.copy()
            Hm = H0.copy()
            Hp[f, i] += e
            Hm[f, i] -= e
            if flags & 32:
                out[f, i] = (oracle_L_pot(w, Hp, flags, lr) - oracle_L_pot(w, Hm, flags, lr)) / (2 * e)
            else:
                out[f, i] = (oracle_L(w, Hp, flags, lr, lp) - oracle_L(w, Hm, flags, lr, lp)) / (2 * e)
    return out


def compare(d, ref, mx=1e-6, l2=1e-6):
    scale = float(np.abs(ref).max())
    em = float(np.abs(d - ref).max()) / scale
    e2 = float(np.linalg.norm(d - ref) / np.linalg.norm(ref))
    say(f"  max/max|ref| {em:.2e}  rel-L2 {e2:.2e}")
    assert em < mx and e2 < l2, (em, e2)


@pytest.mark.parametrize("nr,nphi,nf,flags,gap,lin", [
    (7, 8, 2, 0, 3.0, False),      # odd n_r, two groups, temperature gap
    (10, 16, 1, 4, None, False),   # indirect term through H_a at the source ring
    (6, 8, 3, 1, None, False),     # three groups, own cell dropped
    (6, 8, 2, 4, None, True),      # uniform grid: one-sided own-cell integrals
])
def test_ss_grad_matches_oracle_differences(sg, T, W, nr, nphi, nf, flags, gap, lin):
    say(f"semi-spectral dL/dH {nr}x{nphi} nf={nf} flags={flags} gap={gap} linear={lin}")
    w = W.flaring(seed=nr * 3 + nphi, n_r=nr, n_phi=nphi, p=0.25, gap_w=gap, n_fluids=nf, linear_r=lin)
    if lin:
        flags |= sg.LINEAR_R
    if flags & sg.INDIRECT:
        phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
        w["sigma"] = w["sigma"] * (1 + 0.3 * np.cos(phi - 1.0))[None, None, :]
    lr, lp = lams(w["sigma"].shape, nr + nf)
    _, d = gpu_grad(sg, T, w, flags, lr, lp)
    ref = oracle_fd(w, flags, lr, lp)
    compare(d, ref)


@pytest.mark.parametrize("nr,nphi,nf,flags,gap,lin", [
    (7, 8, 2, 0, 3.0, False),      # odd n_r, two groups, temperature gap
    (6, 8, 3, 1, None, False),     # three groups, own cell dropped
    (6, 8, 2, 0, None, True),      # uniform grid: one-sided own-cell integrals
])
def test_ss_grad_potential_matches_oracle_differences(sg, T, W, nr, nphi, nf, flags, gap, lin):
    """dL/dH(r) of the potential operators (SG_POTENTIAL, Sect. 5.5): central
    differences of the oracle's L = <lam_r, Phi(H)>, one ring and fluid at a
    time, with the own-cell integral's derivative (or without the own cell)."""
    say(f"semi-spectral potential dL/dH {nr}x{nphi} nf={nf} flags={flags} gap={gap} linear={lin}")
    w = W.flaring(seed=nr * 5 + nphi, n_r=nr, n_phi=nphi, p=0.25, gap_w=gap, n_fluids=nf, linear_r=lin)
    flags |= sg.POTENTIAL
    if lin:
        flags |= sg.LINEAR_R
    lr, lp = lams(w["sigma"].shape, nr + 3 * nf)
    _, d = gpu_grad(sg, T, w, flags, lr, lp)
    ref = oracle_fd(w, flags, lr, lp)
    compare(d, ref)


def test_ss_grad_chain_rule_constant_aspect(sg, T, W):
    """H_f = h_f r: sum_i r_i dL/dH_f(r_i) against the oracle's dL/dh_f."""
    nr, nphi, nf = 24, 16, 2
    say(f"semi-spectral dL/dH chain rule {nr}x{nphi} nf={nf}")
    w = W.flaring(seed=4, n_r=nr, n_phi=nphi, p=0.0, n_fluids=nf)
    r = w["r"] if "r" in w else np.exp(np.log(w["r_min"]) + (np.arange(nr) + 0.5) *
                                       np.log(w["r_max"] / w["r_min"]) / nr)
    h = w["H"][:, 0] / r[0]
    w["H"] = h[:, None] * r[None, :]
    lr, lp = lams(w["sigma"].shape, 7)
    _, d = gpu_grad(sg, T, w, 0, lr, lp)
    got = (d * r[None, :]).sum(axis=1)
    sig = w["sigma"].astype(np.float32).astype(np.float64)
    ref = O.adjoint_h(nr, nphi, w["r_min"], w["r_max"], h, sig, lr.astype(np.float64),
                      lp.astype(np.float64))
    say(f"  dL/dh gpu {got}  oracle {ref}")
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-6 * float(np.abs(ref).max()))


def oracle_L_hat(w, H, flags, lr, lp):
    """L = <lam, g(H)> with the oracle's second-order ring-pair sum (and its
    point-mass indirect term with the ring H at every cell)."""
    nf, nr, nphi = w["sigma"].shape
    sig = w["sigma"].astype(np.float32).astype(np.float64)
    gr, gp = O.field_ring_hat(nr, nphi, w["r_min"], w["r_max"], H, sig)
    lr = lr.reshape(nf, -1).astype(np.float64)
    lp = lp.reshape(nf, -1).astype(np.float64)
    L = float(np.sum(lr * gr) + np.sum(lp * gp))
    if flags & 4:
        Hc = np.repeat(H[:, :, None], nphi, axis=2)
        AB = O.indirect(nr, nphi, w["r_min"], w["r_max"], [0.0] * nf, sig, H=Hc)
        ir, ip = O.indirect_field(nr, nphi, AB)
        L += float(np.sum(lr * ir[None, :]) + np.sum(lp * ip[None, :]))
    return L


@pytest.mark.parametrize("nr,nphi,nf,flags,gap", [(5, 8, 1, 0, None), (4, 8, 2, 4, 3.0)])
def test_ss_grad_second_order_matches_oracle_differences(sg, T, W, nr, nphi, nf, flags, gap):
    """dL/dH(r) of second-order operators (the h derivatives of the hat
    weights, integrated near the singular point) against central differences
    of the oracle's second-order L, ring by ring (1e-6 of max|dL/dH|)."""
    say(f"semi-spectral second-order dL/dH {nr}x{nphi} nf={nf} flags={flags} gap={gap}")
    w = W.flaring(seed=nr * 7 + nphi, n_r=nr, n_phi=nphi, p=0.25, gap_w=gap, n_fluids=nf)
    if flags & sg.INDIRECT:
        phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
        w["sigma"] = w["sigma"] * (1 + 0.3 * np.cos(phi - 1.0))[None, None, :]
    lr, lp = lams(w["sigma"].shape, nr + 5 * nf)
    _, d = gpu_grad(sg, T, w, flags | sg.SECOND_ORDER, lr, lp)
    H0 = np.array(w["H"], dtype=np.float64)
    ref = np.zeros_like(H0)
    for f in range(nf):
        for i in range(nr):
            e = 1e-4 * H0[f, i]
            Hp, Hm = H0.copy(), H0.copy()
            Hp[f, i] += e
            Hm[f, i] -= e
            ref[f, i] = (oracle_L_hat(w, Hp, flags, lr, lp) - oracle_L_hat(w, Hm, flags, lr, lp)) / (2 * e)
    compare(d, ref)


def test_ss_grad_second_order_chain_rule_constant_aspect(sg, T, W):
    """H_f = h_f r with second-order operators: sum_i r_i dL/dH_f(r_i)
    against the oracle's dL/dh_f of the second-order offset table (the FFT
    path's model, which these operators equal for H = h r)."""
    nr, nphi, nf = 12, 16, 2
    say(f"semi-spectral second-order dL/dH chain rule {nr}x{nphi} nf={nf}")
    w = W.flaring(seed=5, n_r=nr, n_phi=nphi, p=0.0, n_fluids=nf)
    r = np.exp(np.log(w["r_min"]) + (np.arange(nr) + 0.5) * np.log(w["r_max"] / w["r_min"]) / nr)
    h = w["H"][:, 0] / r[0]
    w["H"] = h[:, None] * r[None, :]
    lr, lp = lams(w["sigma"].shape, 9)
    _, d = gpu_grad(sg, T, w, sg.SECOND_ORDER, lr, lp)
    got = (d * r[None, :]).sum(axis=1)
    sig = w["sigma"].astype(np.float32).astype(np.float64)
    ref = O.adjoint_h(nr, nphi, w["r_min"], w["r_max"], h, sig, lr.astype(np.float64),
                      lp.astype(np.float64), flags=O.SECOND_ORDER)
    say(f"  dL/dh gpu {got}  oracle {ref}")
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-6 * float(np.abs(ref).max()))


def test_ss_grad_directional_full_size(sg, T, W):
    """App. D size (1200 x 2048): a repeated call is identical bit for bit, and
    <dL/dH, dH> agrees with the central difference
    of the GPU forward along a smooth dH.  The forward and its table are
    float, so the difference carries their rounding (a few 1e-4 of the
    derivative at eps = 1e-3, less at larger eps); eps = 4e-3 keeps the
    truncation error below that."""
    say("semi-spectral dL/dH directional derivative 1200x2048")
    w = W.flaring(seed=1, n_r=1200, n_phi=2048, p=0.25, gap_w=40.0, n_fluids=1)
    nr = w["n_r"]
    lr, lp = lams(w["sigma"].shape, 3)
    S, d = gpu_grad(sg, T, w, 0, lr, lp)
    # the ring-pair partials are summed in a fixed order: a second call is identical
    H = torch.tensor(w["H"], dtype=torch.float64, device="cuda")
    d2 = torch.empty_like(H)
    ws = torch.empty(sg.ss_grad_H_workspace_bytes(S.disc), dtype=torch.uint8, device="cuda")
    sg.ss_grad_H(S.disc, H, torch.tensor(lr).cuda(), torch.tensor(lp).cuda(), d2, ws)
    torch.cuda.synchronize()
    assert np.array_equal(d2.cpu().numpy(), d)
    del ws, d2
    u = np.linspace(0.0, 1.0, nr)
    dH = w["H"] * (0.5 + np.sin(7.0 * u))[None, :]
    lr_t, lp_t = torch.tensor(lr).cuda().double(), torch.tensor(lp).cuda().double()

    def L(Hx):
        S.refresh(Hx)
        S.run()
        torch.cuda.synchronize()
        return float((lr_t * S.g_r.double()).sum() + (lp_t * S.g_phi.double()).sum())

    eps = 4e-3
    fd = (L(w["H"] + eps * dH) - L(w["H"] - eps * dH)) / (2 * eps)
    got = float(np.sum(d * dH))
    say(f"  <dL/dH, dH> {got:.8e}  difference {fd:.8e}  rel {abs(got - fd) / abs(fd):.2e}")
    assert abs(got - fd) < 2e-3 * abs(fd)


def test_ss_grad_species_equals_group_disc(sg, T, W):
    """A species disc's dL/dH is that of the disc of its group sums (formed in
    the forward's order)."""
    groups = (0, 1, 1, 0)
    nr, nphi = 11, 16
    say(f"semi-spectral dL/dH species {groups} {nr}x{nphi}")
    w = W.flaring(seed=5, n_r=nr, n_phi=nphi, p=0.25, n_fluids=2)
    rng = np.random.default_rng(6)
    sig = np.zeros((len(groups), nr, nphi), dtype=np.float32)
    for gi in range(2):
        members = [s for s, g in enumerate(groups) if g == gi]
        wts = rng.uniform(0.2, 1.0, (len(members), nr, nphi))
        wts /= wts.sum(axis=0)
        for k, s in enumerate(members):
            sig[s] = (w["sigma"][gi] * wts[k]).astype(np.float32)
    sums = np.zeros((2, nr, nphi), dtype=np.float32)
    for s, g in enumerate(groups):
        sums[g] = sums[g] + sig[s]
    lr, lp = lams((2, nr, nphi), 9)
    H = torch.tensor(w["H"], dtype=torch.float64, device="cuda")
    out = []
    for species, sigma in ((groups, sig), (None, sums)):
        S = T.SemiSpectral(nr, nphi, w["r_min"], w["r_max"], 2, 0, species_group=species)
        S.refresh(w["H"])
        S.sigma.copy_(torch.tensor(sigma))
        dH = torch.empty_like(H)
        ws = torch.empty(sg.ss_grad_H_workspace_bytes(S.disc), dtype=torch.uint8, device="cuda")
        sg.ss_grad_H(S.disc, H, torch.tensor(lr).cuda(), torch.tensor(lp).cuda(), dH, ws)
        torch.cuda.synchronize()
        out.append(dH.cpu().numpy())
    err = float(np.abs(out[0] - out[1]).max() / np.abs(out[1]).max())
    say(f"  max/max|dL/dH| {err:.2e}")
    assert err < 1e-12


def test_ss_grad_rejects(sg, T, W):
    """FFT-path discs (no radial operators) are refused."""
    w = W.bifluid_fft(seed=2, n_r=8, n_phi=8)
    F = T.FFTField([w])
    assert sg.ss_grad_H_workspace_bytes(F.discs[0]) == 0
    H = torch.ones((2, 8), dtype=torch.float64, device="cuda")
    lam = torch.zeros(F.g_r[0].shape, device="cuda")
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        sg.ss_grad_H(F.discs[0], H, lam, lam, torch.empty_like(H), ws)
