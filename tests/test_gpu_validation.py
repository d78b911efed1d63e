"""Validation against closed forms at the paper's resolution (Sect. 4.3): the
razor-thin exponential disc, whose radial acceleration is known exactly
(Freeman's disc): g_r = -2 pi G Sigma_0 y [I0(y) K0(y) - I1(y) K1(y)],
y = r/(2 r_0).  The exact Bessel kernel tends to the razor-thin one as H -> 0,
and the paper finds the relative error levelling off near 1e-4 for small
aspect ratios.  Run on the FFT path (H = h r, q = 1) and on the
semi-spectral path (H constant, q = 0), as the paper does with its two codes.
The comparison uses y in [0.05, 2.5]: the field vanishes at y = 0 (relative
error meaningless there, as the paper notes) and the grid's outer edge at
y = 5 truncates the disc.

With the second-order table (SG_SECOND_ORDER) the discretisation term
drops below the floor and the error is the floor itself, about h: at
h = 1e-4 that is the paper's ~1e-4 level (tested below).

Two parts make up the error against Freeman with the point-sampled table:
  * a continuum floor: the exact kernel describes Gaussian columns of height
    H, Freeman's field a razor-thin disc; with H = h r the two differ by about
    h (1.0 h at h = 0.01, 1.2 h at h = 0.001, measured with a second-order
    evaluation of the continuum field in test_validation_floor.py), so the
    paper's ~1e-4 is out of reach at h = 0.001 for this kernel (it is what
    constant-H runs reach, where h = H / r is far smaller);
  * the discretisation: the cell-centre sums (point masses, own cell
    averaged) converge at first order in du on a log grid, because the ring
    kernel has a 1/X and a log|X| singularity and the linear variation of
    Sigma inside the neighbour cells no longer cancels against it.  At the
    1024 x 2048 grid (du = 0.012) this adds about 2.4e-3 at h = 0.001.
The bounds below follow these two parts (floor + first-order term), and the
convergence test checks the first order itself."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
special = pytest.importorskip("scipy.special")


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


def freeman(r, r0, sig0):
    y = r / (2 * r0)
    # I_n(y) K_n(y) = i_ne(y) k_ne(y): the exponential scalings cancel
    b = special.i0e(y) * special.k0e(y) - special.i1e(y) * special.k1e(y)
    return -2 * np.pi * sig0 * y * b, y


def errors(w, gr):
    r = np.exp(np.log(w["r_min"]) + (np.arange(w["n_r"]) + 0.5) * np.log(w["r_max"] / w["r_min"]) / w["n_r"])
    ref, y = freeman(r, w["r0"], w["sigma0"])
    prof = gr.reshape(w["n_r"], w["n_phi"]).mean(axis=1)
    spread = float(np.abs(gr.reshape(w["n_r"], w["n_phi"]) - prof[:, None]).max() / np.abs(ref).max())
    sel = (y >= 0.05) & (y <= 2.5)
    rel = np.abs(prof[sel] - ref[sel]) / np.abs(ref[sel])
    return float(np.median(rel)), float(rel.max()), spread


@pytest.mark.parametrize("h,med_bar,max_bar", [(0.01, 2e-2, 5e-2), (0.001, 5e-3, 3e-2)])
def test_exponential_disc_fft_path(sg, T, W, h, med_bar, max_bar):
    print(f"exponential disc, FFT path, H = {h} r, 1024x2048", flush=True)
    w = W.exponential(h=h, q=1)
    F = T.FFTField([dict(w, h=[h])])
    F.set_sigma(0, w["sigma"])
    F.run()
    torch.cuda.synchronize()
    med, mx, spread = errors(w, F.g_r[0][0].double().cpu().numpy())
    print(f"  relative error vs Freeman: median {med:.2e} max {mx:.2e}; azimuthal spread {spread:.1e}",
          flush=True)
    assert spread < 1e-5
    assert med < med_bar and mx < max_bar


@pytest.mark.parametrize("H,med_bar,max_bar", [(0.01, 5e-3, 3e-2)])
def test_exponential_disc_semispectral(sg, T, W, H, med_bar, max_bar):
    """The paper's N_r = 1200 (any n_r on this path), constant H (q = 0)."""
    print(f"exponential disc, semi-spectral, H = {H}, 1200x2048", flush=True)
    w = W.exponential(n_r=1200, n_phi=2048, h=H, q=0)
    S = T.SemiSpectral(w["n_r"], w["n_phi"], w["r_min"], w["r_max"], 1)
    S.refresh(w["H"])
    S.release_workspace()
    S.sigma.copy_(torch.tensor(w["sigma"], dtype=torch.float32))
    S.run()
    torch.cuda.synchronize()
    med, mx, spread = errors(w, S.g_r[0].double().cpu().numpy())
    print(f"  relative error vs Freeman: median {med:.2e} max {mx:.2e}; azimuthal spread {spread:.1e}",
          flush=True)
    assert spread < 1e-5
    assert med < med_bar and mx < max_bar


def test_exponential_disc_first_order_convergence(sg, T, W):
    """Halving du and dphi halves the error (first order in du), FFT path,
    H = 0.001 r."""
    meds = []
    for nr, nphi in ((256, 512), (512, 1024), (1024, 2048)):
        w = W.exponential(n_r=nr, n_phi=nphi, h=0.001, q=1)
        F = T.FFTField([dict(w, h=[0.001])])
        F.set_sigma(0, w["sigma"])
        F.run()
        torch.cuda.synchronize()
        med, mx, _ = errors(w, F.g_r[0][0].double().cpu().numpy())
        print(f"  {nr}x{nphi}: median {med:.2e} max {mx:.2e}", flush=True)
        meds.append(med)
    for a, b in zip(meds, meds[1:]):
        assert 1.6 < a / b < 2.5, meds


def test_exponential_disc_second_order_table_reaches_the_floor(sg, T, W):
    """With SG_SECOND_ORDER (hat-weighted table) the discretisation error is
    second order, so at h = 0.001 the error against Freeman falls to the
    continuum floor (about h, test_validation_floor.py) already on the
    coarser grids and stays there (seen 9.8e-4 to 1.0e-3 from 256 x 512 to
    1024 x 2048), where the cell-centre sums sit a first-order term above it
    (3.5e-3 at 1024 x 2048)."""
    meds = []
    for nr, nphi in ((256, 512), (512, 1024), (1024, 2048)):
        w = W.exponential(n_r=nr, n_phi=nphi, h=0.001, q=1)
        F = T.FFTField([dict(w, h=[0.001])], flags=sg.SECOND_ORDER)
        F.set_sigma(0, w["sigma"])
        F.run()
        torch.cuda.synchronize()
        med, mx, spread = errors(w, F.g_r[0][0].double().cpu().numpy())
        print(f"  second order {nr}x{nphi}: median {med:.2e} max {mx:.2e} spread {spread:.1e}", flush=True)
        assert spread < 1e-5
        meds.append(med)
    assert 0.9e-3 < meds[-1] < 1.6e-3, meds
    assert abs(meds[1] / meds[2] - 1) < 0.15, meds


def test_exponential_disc_reaches_the_paper_level_with_the_second_order_table(sg, T, W):
    """The paper's exponential disc levels off near 1e-4 (Sect. 4.2).  With
    H = h r the continuum floor is about h (reading of the validation), so at
    h = 1e-4 the second-order table reaches that level at 1024 x 2048 (seen:
    median 9.6e-5, max 3.1e-4), where the point-sampled table stays a
    first-order term above it (median 3.4e-3).  Across h = 1e-4, 3e-4 and
    1e-3 the median is h itself to within 10 % (seen 0.96 h to 1.0 h): what
    remains is the kernel's finite thickness, not the discretisation."""
    out = {}
    for h in (1e-4, 3e-4, 1e-3):
        for fl in (0, sg.SECOND_ORDER):
            if fl == 0 and h != 1e-4:
                continue
            w = W.exponential(n_r=1024, n_phi=2048, h=h, q=1)
            F = T.FFTField([dict(w, h=[h])], flags=fl)
            F.set_sigma(0, w["sigma"])
            F.run()
            torch.cuda.synchronize()
            med, mx, spread = errors(w, F.g_r[0][0].double().cpu().numpy())
            print(f"  h = {h:g}, {'second-order' if fl else 'point'} table: median {med:.2e} max {mx:.2e}",
                  flush=True)
            assert spread < 1e-5
            out[(h, fl)] = (med, mx)
            del F
    med, mx = out[(1e-4, sg.SECOND_ORDER)]
    assert med < 1.5e-4 and mx < 5e-4, out
    assert out[(1e-4, 0)][0] > 10 * med, out
    for h in (1e-4, 3e-4, 1e-3):
        assert 0.9 < out[(h, sg.SECOND_ORDER)][0] / h < 1.1, out


def test_exponential_disc_semispectral_second_order_reaches_the_paper_level(sg, T, W):
    """The paper's own setting for its ~1e-4 plateau (Sect. 4.2): constant
    H (q = 0) on the semi-spectral path, N_r = 1200.  With the second-order
    operators the median error against Freeman falls to about 1e-4 (seen
    8.3e-5, max 3.1e-4; H / r is below 4e-4 over the compared radii, so the
    continuum floor is not what remains), where the point-sampled operators
    give 2.9e-3."""
    w = W.exponential(n_r=1200, n_phi=2048, h=0.01, q=0)
    out = {}
    for fl in (0, sg.SECOND_ORDER):
        S = T.SemiSpectral(w["n_r"], w["n_phi"], w["r_min"], w["r_max"], 1, fl)
        S.refresh(w["H"])
        S.release_workspace()
        S.sigma.copy_(torch.tensor(w["sigma"], dtype=torch.float32))
        S.run()
        torch.cuda.synchronize()
        med, mx, spread = errors(w, S.g_r[0].double().cpu().numpy())
        print(f"  {'second-order' if fl else 'point'} operators: median {med:.2e} max {mx:.2e}", flush=True)
        assert spread < 1e-5
        out[fl] = (med, mx)
        del S
    med, mx = out[sg.SECOND_ORDER]
    assert med < 1.5e-4 and mx < 5e-4, out
    assert out[0][0] > 10 * med, out


def test_appD_constant_h_error_grows_with_flaring(sg, T, W):
    """App. D: the full FFT method needs H/r constant; on a flaring disc its
    field differs from the semi-spectral reference computed with the true
    H(r), more so the stronger the flaring, while a temperature gap only
    matters near the gap.  Power-law disc Sigma ~ r^-1.5 on [20, 250] AU,
    512 x 1024; FFT path with h = 0.05 against the semi-spectral path with
    H/r = 0.05 (r/100)^p (and with the gap factor)."""
    nr, nphi = 512, 1024
    base = W.flaring(seed=1, n_r=nr, n_phi=nphi, p=0.0)
    sig = base["sigma"].copy()
    r = np.exp(np.log(base["r_min"]) + (np.arange(nr) + 0.5) * np.log(base["r_max"] / base["r_min"]) / nr)
    sig[:] = (r / 100.0)[None, :, None] ** -1.5  # axisymmetric power-law disc
    F = T.FFTField([dict(base, h=[0.05])])
    F.set_sigma(0, sig)
    F.run()
    torch.cuda.synchronize()
    g_fft = F.g_r[0][0].double().cpu().numpy().mean(axis=1)

    def err(p, gap):
        w = W.flaring(seed=1, n_r=nr, n_phi=nphi, p=p, gap_w=gap)
        S = T.SemiSpectral(nr, nphi, w["r_min"], w["r_max"], 1)
        S.refresh(w["H"])
        S.sigma.copy_(torch.tensor(sig, dtype=torch.float32))
        S.run()
        torch.cuda.synchronize()
        g = S.g_r[0].double().cpu().numpy().mean(axis=1)
        rel = np.abs(g_fft - g) / np.abs(g)
        keep = np.abs(g) > 0.05 * np.abs(g).max()  # away from the zero of g_r
        return rel, keep

    med = {}
    for p in (0.125, 0.25, 0.5):
        rel, keep = err(p, None)
        med[p] = float(np.median(rel[keep]))
        print(f"  flaring p = {p}: median relative difference {med[p]:.2e}, max {rel[keep].max():.2e}",
              flush=True)
    assert med[0.125] < med[0.25] < med[0.5]
    rel, keep = err(0.0, 10.0)
    near = keep & (np.abs(r - 100.0) < 30.0)
    far = keep & (np.abs(r - 100.0) > 60.0)
    print(f"  gap w = 10: max near the gap {rel[near].max():.2e}, median far from it {np.median(rel[far]):.2e}",
          flush=True)
    assert rel[near].max() > 10 * np.median(rel[far])
