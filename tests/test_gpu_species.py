"""Species sharing kernel groups (n_species > 0): the paper's multi-fluid
proposal (Sect. 5.2) of one kernel per scale-height group, with each group's
source density the sum of its species.  Checked through the C ABI: bitwise
equal to the two-fluid disc whose dust density is the float sum of the dust
species (the library adds the species in index order while reading them),
and against the pairwise oracle on the group sums (1e-5 relative RMS), on the
FFT path and the semi-spectral path."""
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


def species_of(w, groups, seed):
    """Splits the workload's densities into species: each group's density is
    shared out over its species with seeded positive weights."""
    rng = np.random.default_rng(seed)
    sig = np.zeros((len(groups),) + w["sigma"].shape[1:], dtype=np.float32)
    for gi in range(w["sigma"].shape[0]):
        members = [s for s, g in enumerate(groups) if g == gi]
        wts = rng.uniform(0.2, 1.0, (len(members),) + w["sigma"].shape[1:])
        wts /= wts.sum(axis=0)
        for k, s in enumerate(members):
            sig[s] = (w["sigma"][gi] * wts[k]).astype(np.float32)
    return sig


def group_sums(sig, groups, nf):
    out = np.zeros((nf,) + sig.shape[1:], dtype=np.float32)
    for s, g in enumerate(groups):
        out[g] = out[g] + sig[s]  # float32, species order
    return out


@pytest.mark.parametrize("groups,nr,nphi", [((0, 1, 1), 32, 64), ((1, 0, 1, 0, 1), 16, 32), ((0, 0), 8, 16)])
def test_species_fft_path(sg, T, W, groups, nr, nphi):
    print(f"species {groups} fft path {nr}x{nphi}", flush=True)
    nf = max(groups) + 1 if max(groups) > 0 else 2
    w = W.bifluid_fft(seed=nr + len(groups), n_r=nr, n_phi=nphi)
    sig = species_of(w, groups, nr)
    spec = dict(w, species_group=list(groups))
    Fs = T.FFTField([spec])
    Fs.sigma[0].copy_(torch.tensor(sig))
    Fs.run()
    Fg = T.FFTField([w])
    sums = group_sums(sig, groups, 2)
    Fg.sigma[0].copy_(torch.tensor(sums))
    Fg.run()
    torch.cuda.synchronize()
    for a, b in ((Fs.g_r[0], Fg.g_r[0]), (Fs.g_phi[0], Fg.g_phi[0])):
        assert torch.equal(a, b)
    rr, rp = O.field_pairwise(nr, nphi, w["r_min"], w["r_max"], w["h"], sums.astype(np.float64))
    gr = Fs.g_r[0].double().cpu().numpy().reshape(2, -1)
    gp = Fs.g_phi[0].double().cpu().numpy().reshape(2, -1)
    for f in range(nf):
        er, ep = rel_rms(gr[f], rr[f]), rel_rms(gp[f], rp[f])
        print(f"  group {f}: rel-RMS {er:.2e} {ep:.2e}", flush=True)
        assert er < 1e-5 and ep < 1e-5


def test_species_semispectral_with_indirect(sg, T, W):
    print("species (0, 1, 0, 1) semi-spectral with the indirect term", flush=True)
    groups = (0, 1, 0, 1)
    w = W.flaring(seed=4, n_r=21, n_phi=32, p=0.25, n_fluids=2)
    phi = (np.arange(32) + 0.5) * 2 * np.pi / 32
    w["sigma"] = w["sigma"] * (1 + 0.3 * np.cos(phi - 2.0))[None, None, :]
    sig = species_of(w, groups, 3)
    S = T.SemiSpectral(21, 32, w["r_min"], w["r_max"], 2, flags=sg.INDIRECT, species_group=groups)
    S.refresh(w["H"])
    S.sigma.copy_(torch.tensor(sig))
    S.run()
    G = T.SemiSpectral(21, 32, w["r_min"], w["r_max"], 2, flags=sg.INDIRECT)
    G.refresh(w["H"])
    sums = group_sums(sig, groups, 2)
    G.sigma.copy_(torch.tensor(sums))
    G.run()
    torch.cuda.synchronize()
    assert torch.equal(S.g_r, G.g_r) and torch.equal(S.g_phi, G.g_phi)
    Hc = np.repeat(w["H"][:, :, None], 32, axis=2)
    s64 = sums.astype(np.float64)
    rr, rp = O.field_pairwise(21, 32, w["r_min"], w["r_max"], [0.0, 0.0], s64, H=Hc)
    ir, ip = O.indirect_field(21, 32, O.indirect(21, 32, w["r_min"], w["r_max"], [0.0, 0.0], s64, H=Hc))
    gr = S.g_r.double().cpu().numpy().reshape(2, -1)
    gp = S.g_phi.double().cpu().numpy().reshape(2, -1)
    for f in range(2):
        er, ep = rel_rms(gr[f], rr[f] + ir), rel_rms(gp[f], rp[f] + ip)
        print(f"  group {f}: rel-RMS {er:.2e} {ep:.2e}", flush=True)
        assert er < 1e-5 and ep < 1e-5


def adjoint(sg, disc, lam_r, lam_p, dsig_shape, n_dh):
    ds = torch.empty(dsig_shape, dtype=torch.float32, device="cuda")
    dh = torch.empty(n_dh, dtype=torch.float64, device="cuda") if n_dh else None
    ws = torch.empty(sg.field_adjoint_workspace_bytes(disc), dtype=torch.uint8, device="cuda")
    sg.field_adjoint(disc, lam_r, lam_p, ds, dh, ws)
    torch.cuda.synchronize()
    return ds, dh


def test_species_adjoint_fft_path(sg, T, W):
    """Species adjoint: every species gets its group's dL/dSigma and dL/dh is
    that of the group densities (bitwise equal to the group disc's adjoint,
    whose own parity with the oracle is tested elsewhere), plus the transpose
    identity <lam, g(Sigma_species)> = sum_s <dL/dSigma_s, Sigma_s> (1e-5)."""
    groups = (0, 1, 1, 0, 1)
    nr, nphi = 32, 64
    print(f"species adjoint {groups} fft path {nr}x{nphi}", flush=True)
    w = W.bifluid_fft(seed=9, n_r=nr, n_phi=nphi)
    sig = species_of(w, groups, 5)
    Fs = T.FFTField([dict(w, species_group=list(groups))], flags=sg.WITH_DH)
    Fs.sigma[0].copy_(torch.tensor(sig))
    Fs.run()
    Fg = T.FFTField([w], flags=sg.WITH_DH)
    sums = group_sums(sig, groups, 2)
    Fg.sigma[0].copy_(torch.tensor(sums))
    torch.cuda.synchronize()
    gen = torch.Generator(device="cpu").manual_seed(11)
    lam_r = torch.randn((2, nr, nphi), generator=gen).cuda()
    lam_p = torch.randn((2, nr, nphi), generator=gen).cuda()
    ds, dh = adjoint(sg, Fs.discs[0], lam_r, lam_p, (len(groups), nr, nphi), 2)
    dg, dhg = adjoint(sg, Fg.discs[0], lam_r, lam_p, (2, nr, nphi), 2)
    for s, g in enumerate(groups):
        assert torch.equal(ds[s], dg[g]), s
    assert torch.equal(dh, dhg), (dh, dhg)
    lhs = float((lam_r.double() * Fs.g_r[0].double()).sum() + (lam_p.double() * Fs.g_phi[0].double()).sum())
    rhs = float((ds.double() * Fs.sigma[0].double()).sum())
    print(f"  <lam, g> {lhs:.8e}  <dL/dSigma, Sigma> {rhs:.8e}", flush=True)
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


def test_species_adjoint_semispectral(sg, T, W):
    """As above on a semi-spectral disc with the indirect term (dL/dSigma)."""
    groups = (1, 0, 1, 1)
    nr, nphi = 21, 32
    print(f"species adjoint {groups} semi-spectral {nr}x{nphi}", flush=True)
    w = W.flaring(seed=6, n_r=nr, n_phi=nphi, p=0.25, n_fluids=2)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    w["sigma"] = w["sigma"] * (1 + 0.3 * np.cos(phi - 2.0))[None, None, :]
    sig = species_of(w, groups, 8)
    S = T.SemiSpectral(nr, nphi, w["r_min"], w["r_max"], 2, flags=sg.INDIRECT, species_group=groups)
    S.refresh(w["H"])
    S.sigma.copy_(torch.tensor(sig))
    S.run()
    G = T.SemiSpectral(nr, nphi, w["r_min"], w["r_max"], 2, flags=sg.INDIRECT)
    G.refresh(w["H"])
    torch.cuda.synchronize()
    gen = torch.Generator(device="cpu").manual_seed(12)
    lam_r = torch.randn((2, nr, nphi), generator=gen).cuda()
    lam_p = torch.randn((2, nr, nphi), generator=gen).cuda()
    ds, _ = adjoint(sg, S.disc, lam_r, lam_p, (len(groups), nr, nphi), 0)
    dg, _ = adjoint(sg, G.disc, lam_r, lam_p, (2, nr, nphi), 0)
    for s, g in enumerate(groups):
        assert torch.equal(ds[s], dg[g]), s
    lhs = float((lam_r.double() * S.g_r.double()).sum() + (lam_p.double() * S.g_phi.double()).sum())
    rhs = float((ds.double() * S.sigma.double()).sum())
    print(f"  <lam, g> {lhs:.8e}  <dL/dSigma, Sigma> {rhs:.8e}", flush=True)
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)
