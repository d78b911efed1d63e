"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/sg.h, sizes are computed on the host and
invalid arguments are rejected before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sg.h")


@pytest.fixture(scope="module")
def sg():
    libp = os.path.join(ROOT, "paper_2506_10812_amd", "libsg.so")
    csrc = os.path.join(ROOT, "paper_2506_10812_amd", "csrc")
    newest = max(os.path.getmtime(os.path.join(csrc, f)) for f in os.listdir(csrc))
    if not os.path.exists(libp) or os.path.getmtime(libp) < newest:
        from paper_2506_10812_amd import build
        build.build()
    import paper_2506_10812_amd as m
    return m


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_four_paths():
    names = declared_functions()
    for n in ("sg_kernel_table", "sg_field_direct", "sg_field_fft", "sg_field_adjoint"):
        assert n in names


def test_library_exports_every_declared_symbol(sg):
    lib = ctypes.CDLL(sg.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(sg.EXPORTED)


def test_status_strings(sg):
    for s in range(7):
        assert sg.status_string(s).startswith("SG_")
    assert sg.version() >= 1


def test_table_size_is_host_computable(sg):
    g = sg.grid(1024, 2048, 0.2, 5.0)
    f = sg.fluids([0.05, 0.005])
    nb = sg.kernel_table_bytes(g, f, 0)
    # four ordered pairs x two components x (n_r+1)(n_phi/2+2) complex64 spectra
    # (columns 0 .. n_phi/2 and the pair column) dominate
    spec = 4 * 2 * 1025 * 1026 * 8
    assert spec < nb < spec + 64 * 1024
    nb_dh = sg.kernel_table_bytes(g, f, sg.WITH_DH)
    assert nb_dh - nb >= 2 * (4 * 2 * 1025 * 1025 * 8)  # d/dh_a and d/dh_b spectra
    assert sg.kernel_table_workspace_bytes(g, f, 0) > 0


@pytest.mark.parametrize("nr,nphi", [(3, 8), (8, 12), (1, 8), (4096, 8), (8, 2), (8, 4096)])
def test_fft_path_rejects_unsupported_grids(sg, nr, nphi):
    g = sg.grid(nr, nphi, 0.2, 5.0)
    f = sg.fluids([0.05])
    assert sg.kernel_table_bytes(g, f, 0) == 0
    st = sg.lib().sg_kernel_table(ctypes.byref(g), ctypes.byref(f), 0, ctypes.c_void_p(256),
                                  ctypes.c_void_p(512), 1 << 40, None)
    assert st == sg.ERR_UNSUPPORTED


@pytest.mark.parametrize("h,rmin,rmax", [([0.0], 0.2, 5.0), ([-1.0], 0.2, 5.0),
                                         ([float("nan")], 0.2, 5.0), ([0.05], 0.0, 5.0),
                                         ([0.05], 5.0, 0.2)])
def test_invalid_physics_arguments(sg, h, rmin, rmax):
    g = sg.grid(16, 32, rmin, rmax)
    f = sg.fluids(h)
    st = sg.lib().sg_kernel_table(ctypes.byref(g), ctypes.byref(f), 0, ctypes.c_void_p(256),
                                  ctypes.c_void_p(512), 1 << 40, None)
    assert st == sg.ERR_ARG


def test_workspace_checks_happen_before_launch(sg):
    g = sg.grid(16, 32, 0.2, 5.0)
    f = sg.fluids([0.05])
    st = sg.lib().sg_kernel_table(ctypes.byref(g), ctypes.byref(f), 0, ctypes.c_void_p(256),
                                  ctypes.c_void_p(512), 16, None)
    assert st == sg.ERR_WORKSPACE
    d = sg.Disc(g, f, 0, 0, 256, 512, 768, 1024)
    arr = (sg.Disc * 1)(d)
    need = sg.field_fft_workspace_bytes([d])
    assert need > 0
    assert sg.lib().sg_field_fft(arr, 1, ctypes.c_void_p(2048), need - 1, None) == sg.ERR_WORKSPACE
    assert sg.lib().sg_field_fft(arr, 0, ctypes.c_void_p(2048), need, None) == sg.ERR_ARG
    assert sg.lib().sg_field_fft(None, 1, ctypes.c_void_p(2048), need, None) == sg.ERR_ARG
    d.sigma = None
    arr = (sg.Disc * 1)(d)
    assert sg.lib().sg_field_fft(arr, 1, ctypes.c_void_p(2048), need, None) == sg.ERR_ARG


def test_direct_validation(sg):
    g = sg.grid(5, 7, 0.2, 5.0)
    need = sg.field_direct_workspace_bytes(g, 2, sg.F64, False)
    assert need > 0
    L = sg.lib()
    h = (ctypes.c_double * 5)(0.05, 0.01, 0.02, 0.03, 0.04)
    hp = ctypes.cast(h, ctypes.POINTER(ctypes.c_double))
    # bad dtype, bad fluid count (1 to 4 scale-height groups), missing h, bad flag, small workspace
    assert L.sg_field_direct(ctypes.byref(g), 2, hp, 256, None, 512, 768, 7, 0, 1024, need, None) == sg.ERR_ARG
    assert L.sg_field_direct(ctypes.byref(g), 5, hp, 256, None, 512, 768, sg.F64, 0, 1024, need, None) == sg.ERR_ARG
    assert L.sg_field_direct(ctypes.byref(g), 0, hp, 256, None, 512, 768, sg.F64, 0, 1024, need, None) == sg.ERR_ARG
    assert sg.field_direct_workspace_bytes(g, 4, sg.F64, False) > need
    assert sg.field_direct_workspace_bytes(g, 5, sg.F64, False) == 0
    assert sg.potential_direct_workspace_bytes(g, 4, sg.F32, True) > 0
    assert sg.potential_direct_workspace_bytes(g, 5, sg.F32, True) == 0
    assert L.sg_hsg(10, 5, 256, 512, 768, None) == sg.ERR_ARG
    assert L.sg_field_direct(ctypes.byref(g), 2, None, 256, None, 512, 768, sg.F64, 0, 1024, need, None) == sg.ERR_ARG
    assert L.sg_field_direct(ctypes.byref(g), 2, hp, 256, None, 512, 768, sg.F64, sg.WITH_DH, 1024, need, None) == sg.ERR_ARG
    assert L.sg_field_direct(ctypes.byref(g), 2, hp, 256, None, 512, 768, sg.F64, 0, 1024, need - 1, None) == sg.ERR_WORKSPACE
    big = sg.grid(1 << 14, 1 << 13, 0.2, 5.0)
    assert sg.field_direct_workspace_bytes(big, 1, sg.F32, False) == 0


def test_second_order_flag_combinations(sg):
    """SG_SECOND_ORDER changes the table's values, not its layout (with or
    without d/dh spectra); it cannot be combined with the own-cell switch,
    and the direct sums do not take it (the semi-spectral tables: see
    test_semispectral_sizes_and_validation)."""
    g = sg.grid(16, 32, 0.2, 5.0)
    f = sg.fluids([0.05, 0.005])
    L = sg.lib()
    nb = sg.kernel_table_bytes(g, f, 0)
    assert sg.kernel_table_bytes(g, f, sg.SECOND_ORDER) == nb
    assert sg.kernel_table_bytes(g, f, sg.SECOND_ORDER | sg.INDIRECT) == nb
    assert sg.kernel_table_bytes(g, f, sg.SECOND_ORDER | sg.WITH_DH) == sg.kernel_table_bytes(g, f, sg.WITH_DH)
    assert sg.kernel_table_workspace_bytes(g, f, sg.SECOND_ORDER) > 0
    for bad in (sg.SECOND_ORDER | sg.SELF_CELL_EXCLUDE, sg.SECOND_ORDER | sg.SELF_CELL_EXCLUDE | sg.WITH_DH):
        assert sg.kernel_table_bytes(g, f, bad) == 0
        assert sg.kernel_table_workspace_bytes(g, f, bad) == 0
        st = L.sg_kernel_table(ctypes.byref(g), ctypes.byref(f), bad, ctypes.c_void_p(256),
                               ctypes.c_void_p(512), 1 << 40, None)
        assert st == sg.ERR_UNSUPPORTED
        d = sg.Disc(g, f, bad, 0, 256, 512, 768, 1024)
        assert sg.field_fft_workspace_bytes([d]) == 0
    d = sg.Disc(g, f, sg.SECOND_ORDER, 0, 256, 512, 768, 1024)
    assert sg.field_fft_workspace_bytes([d]) == sg.field_fft_workspace_bytes([sg.Disc(g, f, 0, 0, 256, 512, 768, 1024)])
    need = sg.field_direct_workspace_bytes(g, 1, sg.F64, False)
    h = (ctypes.c_double * 1)(0.05)
    hp = ctypes.cast(h, ctypes.POINTER(ctypes.c_double))
    assert L.sg_field_direct(ctypes.byref(g), 1, hp, 256, None, 512, 768, sg.F64, sg.SECOND_ORDER, 1024, need,
                             None) == sg.ERR_ARG


def test_adjoint_needs_dh_table(sg):
    g = sg.grid(16, 32, 0.2, 5.0)
    f = sg.fluids([0.05])
    d = sg.Disc(g, f, 0, 0, 256, 512, 768, 1024)
    need = sg.field_adjoint_workspace_bytes(d)
    assert need > 0
    st = sg.lib().sg_field_adjoint(ctypes.byref(d), 256, 512, 768, 1024, 2048, need, None)
    assert st == sg.ERR_TABLE


def test_semispectral_sizes_and_validation(sg):
    """sg_ss_table sizes are host-computable for any n_r; unsupported grids,
    bad flags and short workspaces are refused before any launch; semi-spectral
    discs pass the FFT-path checks with their own grid rules."""
    L = sg.lib()
    for nr in (1, 2, 37, 1200, 2048):
        g = sg.grid(nr, 64, 20.0, 250.0)
        nrt = nr + (nr & 1)
        core = 33 * 4 * nr * nrt * 8
        nb = sg.ss_table_bytes(g, 2, sg.SS_FULL)
        assert core < nb < core + 4096, (nr, nb)
        assert sg.ss_table_workspace_bytes(g, 2) > 0
    for nr, nphi in ((2049, 64), (16, 2), (16, 12), (16, 4096), (0, 64)):
        assert sg.ss_table_bytes(sg.grid(nr, nphi, 20.0, 250.0), 1) == 0
    assert sg.ss_table_bytes(sg.grid(16, 64, 20.0, 250.0), 1, sg.WITH_DH) == 0
    g = sg.grid(37, 32, 20.0, 250.0)
    need = sg.ss_table_workspace_bytes(g, 2)
    call = lambda nf, H, flags, tab, ws, n: L.sg_ss_table(ctypes.byref(g), nf, H, flags, tab, ws, n, None)
    assert call(2, 256, 0, 512, 1024, need - 1) == sg.ERR_WORKSPACE
    assert call(2, None, 0, 512, 1024, need) == sg.ERR_ARG
    assert call(5, 256, 0, 512, 1024, need) == sg.ERR_ARG
    # up to four scale-height groups on this path (n_r <= 1024 beyond two)
    assert sg.ss_table_bytes(g, 4) > 2 * sg.ss_table_bytes(g, 2)
    assert sg.ss_table_bytes(sg.grid(1025, 64, 20.0, 250.0), 3) == 0
    assert sg.ss_table_bytes(sg.grid(1025, 64, 20.0, 250.0), 2) > 0
    assert call(2, 256, sg.WITH_DH, 512, 1024, need) == sg.ERR_ARG
    assert call(2, 256, sg.POTENTIAL | sg.INDIRECT, 512, 1024, need) == sg.ERR_ARG
    assert call(2, 256, 0, 520, 1024, need) == sg.ERR_ARG  # table alignment
    bad = sg.grid(37, 48, 20.0, 250.0)
    assert L.sg_ss_table(ctypes.byref(bad), 1, 256, 0, 512, 1024, 1 << 40, None) == sg.ERR_UNSUPPORTED
    # discs: odd n_r passes only with SG_SEMI_SPECTRAL; h is not read
    f = sg.fluids([0.05, 0.01])
    f.h[0] = -1.0
    d = sg.Disc(g, f, sg.SEMI_SPECTRAL, 0, 256, 512, 768, 1024)
    assert sg.field_fft_workspace_bytes([d]) > 0
    d.flags = 0
    assert sg.field_fft_workspace_bytes([d]) == 0
    d.flags = sg.SEMI_SPECTRAL | sg.WITH_DH
    assert sg.field_fft_workspace_bytes([d]) == 0
    d.flags = sg.SEMI_SPECTRAL | sg.INDIRECT | sg.SELF_CELL_EXCLUDE
    assert sg.field_fft_workspace_bytes([d]) > 0
    # semi-spectral adjoint: dL/dSigma only
    assert sg.field_adjoint_workspace_bytes(d) > 0
    assert L.sg_field_adjoint(ctypes.byref(d), 256, 512, 768, 4096, 2048, 1 << 30, None) == sg.ERR_UNSUPPORTED
    # dL/dH(r): semi-spectral discs (field or potential operators, species too)
    need = sg.ss_grad_H_workspace_bytes(d)
    assert need > 0
    G = L.sg_ss_grad_H
    assert G(ctypes.byref(d), None, 512, 768, 4096, 8192, need, None) == sg.ERR_ARG
    assert G(ctypes.byref(d), 256, 512, 768, 4096, 8192, need - 1, None) == sg.ERR_WORKSPACE
    assert G(ctypes.byref(d), 256, 512, 768, 4096, 8200, need, None) == sg.ERR_WORKSPACE
    d.flags = sg.SEMI_SPECTRAL | sg.POTENTIAL
    assert sg.ss_grad_H_workspace_bytes(d) == need
    # second-order operators: solve, dL/dSigma and dL/dH
    d.flags = sg.SEMI_SPECTRAL | sg.SECOND_ORDER
    assert sg.field_fft_workspace_bytes([d]) > 0
    assert sg.ss_grad_H_workspace_bytes(d) == need
    for bad in (sg.POTENTIAL, sg.LINEAR_R, sg.SELF_CELL_EXCLUDE):
        d.flags = sg.SEMI_SPECTRAL | sg.SECOND_ORDER | bad
        assert sg.field_fft_workspace_bytes([d]) == 0
    gs = sg.grid(16, 32, 20.0, 250.0)
    assert sg.ss_table_bytes(gs, 1, sg.SECOND_ORDER) == sg.ss_table_bytes(gs, 1, 0) > 0
    for bad in (sg.POTENTIAL, sg.LINEAR_R, sg.SELF_CELL_EXCLUDE):
        assert sg.ss_table_bytes(gs, 1, sg.SECOND_ORDER | bad) == 0
    fft = sg.make_disc(sg.grid(16, 32, 0.2, 5.0), sg.fluids([0.05]), 0, 256, 512, 768, 1024)
    assert sg.ss_grad_H_workspace_bytes(fft) == 0
    assert G(ctypes.byref(fft), 256, 512, 768, 4096, 8192, 1 << 30, None) == sg.ERR_UNSUPPORTED
    d.flags = sg.SEMI_SPECTRAL
    base = sg.ss_grad_H_workspace_bytes(d)
    d.n_species = 2
    d.species_group[0], d.species_group[1] = 0, 1
    assert sg.field_fft_workspace_bytes([d]) > 0
    # species discs add their group densities (2 x 37 x 32 floats, 256-aligned)
    assert sg.ss_grad_H_workspace_bytes(d) == base + (2 * 37 * 32 * 4 + 255) // 256 * 256


def test_struct_layouts_match_the_header(sg, tmp_path):
    """The ctypes mirrors of sg_grid, sg_fluids, sg_disc and sg_tune_result
    have the C layout (sizes and field offsets from a program built against
    include/sg.h with the host compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    fields = {"sg_grid": ("n_r", "n_phi", "r_min", "r_max"),
              "sg_fluids": ("n_fluids", "h"),
              "sg_disc": ("grid", "fluids", "flags", "n_species", "sigma", "g_r", "g_phi", "table",
                          "species_group"),
              "sg_tune_result": ("pass", "length", "cluster", "rel_best", "ms_best")}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for t, fs in fields.items():
        lines.append(f'printf("{t} sizeof %zu\\n", sizeof({t}));')
        for f in fs:
            lines.append(f'printf("{t} {f} %zu\\n", offsetof({t}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, str(src), "-o", str(exe)])
    got = {}
    for ln in subprocess.check_output([str(exe)], text=True).splitlines():
        t, f, v = ln.split()
        got[(t, f)] = int(v)
    mirror = {"sg_grid": sg.Grid, "sg_fluids": sg.Fluids, "sg_disc": sg.Disc, "sg_tune_result": sg.TuneResult}
    for t, cls in mirror.items():
        assert got[(t, "sizeof")] == ctypes.sizeof(cls), t
        for f in fields[t]:
            name = "pass_" if f == "pass" else f
            assert got[(t, f)] == getattr(cls, name).offset, (t, f)


def test_species_validation(sg):
    g = sg.grid(16, 32, 0.2, 5.0)
    f = sg.fluids([0.05, 0.005])
    ok = sg.make_disc(g, f, 0, 256, 512, 768, 1024, species_group=[0, 1, 1])
    assert ok.n_species == 3 and sg.field_fft_workspace_bytes([ok]) > 0
    assert sg.field_fft_workspace_bytes([sg.make_disc(g, f, 0, 256, 512, 768, 1024, [0, 2])]) == 0
    many = sg.make_disc(g, f, 0, 256, 512, 768, 1024, [0] * 8)
    assert sg.field_fft_workspace_bytes([many]) > 0
    many.n_species = 9
    assert sg.field_fft_workspace_bytes([many]) == 0
    many.n_species = -1
    assert sg.field_fft_workspace_bytes([many]) == 0
    one = sg.make_disc(g, sg.fluids([0.05]), 0, 256, 512, 768, 1024, [0, 1])
    assert sg.field_fft_workspace_bytes([one]) == 0
    # species adjoint: the group run's workspace plus the group densities and
    # the group dL/dSigma (2 x 16 x 32 floats each, 256-byte aligned)
    grp = sg.make_disc(g, f, 0, 256, 512, 768, 1024)
    assert sg.field_adjoint_workspace_bytes(ok) == sg.field_adjoint_workspace_bytes(grp) + 2 * 4096
    assert sg.lib().sg_field_adjoint(ctypes.byref(ok), 256, 512, None, None, 2048, 1 << 30,
                                     None) == sg.ERR_ARG
    assert sg.lib().sg_field_adjoint(ctypes.byref(ok), 256, 512, 768, None, 2048,
                                     sg.field_adjoint_workspace_bytes(ok) - 1, None) == sg.ERR_WORKSPACE



def test_semispectral_band_sizes(sg):
    """Banded modes: m >= 1 keeps |i - i'| <= w_m = ceil(30 ln 2 / (m du)) and is
    stored as 2 w_m + 1 diagonals when 4 w_m + 2 <= n_r; SG_SS_FULL and coarse
    grids keep every mode whole."""
    import math
    for nr, nphi, nf, rmin, rmax in ((1200, 2048, 1, 20.0, 250.0), (1024, 2048, 2, 0.2, 5.0),
                                     (256, 128, 2, 20.0, 250.0), (37, 32, 2, 20.0, 250.0)):
        g = sg.grid(nr, nphi, rmin, rmax)
        du = math.log(rmax / rmin) / nr
        nrt = nr + (nr & 1)
        elems = 0
        for m in range(nphi // 2 + 1):
            w = nr - 1 if m == 0 else min(nr - 1, math.ceil(30 * math.log(2) / (m * du)))
            elems += nf * nf * ((2 * w + 1) if 4 * w + 2 <= nr else nr) * nrt
        full = (nphi // 2 + 1) * nf * nf * nr * nrt
        nb = sg.ss_table_bytes(g, nf)
        nbf = sg.ss_table_bytes(g, nf, sg.SS_FULL)
        assert 8 * elems < nb < 8 * elems + 64 * 1024, (nr, nphi)
        assert 8 * full < nbf < 8 * full + 64 * 1024, (nr, nphi)
        if nr >= 256:
            assert nb < nbf
    # the App. D gas disc: about a tenth of the full operators
    g = sg.grid(1200, 2048, 20.0, 250.0)
    assert sg.ss_table_bytes(g, 1) < 0.15 * sg.ss_table_bytes(g, 1, sg.SS_FULL)


def test_fft_path_group_limits(sg):
    """One to four scale-height groups on the FFT path; beyond two the column
    pass needs n_r <= 1024; the adjoint takes every group count the forward
    takes."""
    g = sg.grid(1024, 2048, 0.2, 5.0)
    nb2 = sg.kernel_table_bytes(g, sg.fluids([0.05, 0.005]), 0)
    nb4 = sg.kernel_table_bytes(g, sg.fluids([0.05, 0.005, 0.02, 0.01]), 0)
    assert nb4 > 3.9 * nb2  # 16 ordered pairs against 4
    assert sg.kernel_table_bytes(sg.grid(2048, 64, 0.2, 5.0), sg.fluids([0.05, 0.005, 0.02]), 0) == 0
    assert sg.kernel_table_bytes(sg.grid(2048, 64, 0.2, 5.0), sg.fluids([0.05, 0.005]), 0) > 0
    f5 = sg.Fluids(5, 0, (ctypes.c_double * 4)(0.05, 0.05, 0.05, 0.05))
    assert sg.kernel_table_bytes(g, f5, 0) == 0
    d3 = sg.make_disc(sg.grid(16, 32, 0.2, 5.0), sg.fluids([0.05, 0.01, 0.02]), 0, 256, 512, 768, 1024)
    assert sg.field_fft_workspace_bytes([d3]) > 0
    assert sg.field_adjoint_workspace_bytes(d3) > 0
    d3big = sg.make_disc(sg.grid(2048, 32, 0.2, 5.0), sg.fluids([0.05, 0.01, 0.02]), 0, 256, 512, 768, 1024)
    assert sg.field_adjoint_workspace_bytes(d3big) == 0
    assert sg.lib().sg_field_adjoint(ctypes.byref(d3big), 256, 512, 768, None, 2048, 1 << 30,
                                     None) == sg.ERR_UNSUPPORTED


def test_noalloc_direct_refuses_oversized_calls_before_device_work(sg):
    """sg_field_direct_noalloc checks its workspace need against the static
    scratch on the host: two float fluids at 1024 x 2048 (96 MiB) are refused
    with SG_ERR_SCRATCH, one fluid (48 MiB) fits; invalid arguments come
    back as SG_ERR_ARG.  No GPU is touched (the pointers are never used)."""
    g = sg.grid(1024, 2048, 0.2, 5.0)
    h = (ctypes.c_double * 4)(0.05, 0.005, 0.0, 0.0)
    hp = ctypes.cast(h, ctypes.POINTER(ctypes.c_double))
    fake = ctypes.c_void_p(256)
    assert sg.field_direct_workspace_bytes(g, 1, sg.F32, False) <= sg.NOALLOC_SCRATCH_BYTES
    st = sg.lib().sg_field_direct_noalloc(ctypes.byref(g), 2, hp, fake, None, fake, fake, sg.F32, 0, None)
    assert st == sg.ERR_SCRATCH
    st = sg.lib().sg_field_direct_noalloc(ctypes.byref(g), 2, hp, None, None, fake, fake, sg.F32, 0, None)
    assert st == sg.ERR_ARG
