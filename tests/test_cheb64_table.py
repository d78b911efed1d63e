"""The library's build-time Chebyshev table (csrc/gen_cheb64.cpp) on the CPU.

The generator is compiled and run here; its coefficients, summed by the
same Clenshaw recurrence and interval mapping as the device branch
(x = m 2^e, interval e, t = 4 m - 3), are checked against the oracle's F,
F' and G0 (themselves pinned to 40-digit Bessel values) at 600 points of
[1/2, 32), interval edges included: 2e-15 relative; and the last kept
coefficient of every interval is below 1e-17 of that interval's largest, so
the dropped tail is below double rounding."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEN = os.path.join(ROOT, "paper_2506_10812_amd", "csrc", "gen_cheb64.cpp")


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    d = tmp_path_factory.mktemp("cheb")
    exe = str(d / "gen")
    subprocess.check_call(["g++", "-O2", "-std=c++17", GEN, "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    ni = int(re.search(r"#define SG_CHEB_NI (\d+)", out).group(1))
    m = int(re.search(r"#define SG_CHEB_M (\d+)", out).group(1))
    arrs = re.findall(r"\{\n(.*?)\};", out, re.S)
    cf = np.array([float(v) for v in arrs[0].replace(",", " ").split()]).reshape(ni, m)
    cd = np.array([float(v) for v in arrs[1].replace(",", " ").split()]).reshape(ni, m)
    cg = np.array([float(v) for v in arrs[2].replace(",", " ").split()]).reshape(ni, m)
    return cf, cd, cg


def clenshaw(x, c):
    mant, e = np.frexp(x)
    k = min(max(int(e), 0), c.shape[0] - 1)
    t = 4.0 * mant - 3.0
    b1 = b2 = 0.0
    for j in range(c.shape[1] - 1, 0, -1):
        b1, b2 = 2.0 * t * b1 - b2 + c[k, j], b1
    return t * b1 - b2 + c[k, 0]


def test_chebyshev_table_matches_the_oracle(table):
    cf, cd, cg = table
    assert cf.shape == cd.shape == cg.shape == (6, 27)
    edges = np.array([0.5, 1.0, 2.0, 4.0, 8.0, 16.0])
    x = np.concatenate([np.geomspace(0.5, 32.0, 580, endpoint=False), edges,
                        np.nextafter(edges[1:], 0.0), np.nextafter(32.0, 0.0)[None]])
    F = np.array([clenshaw(v, cf) for v in x])
    dF = np.array([clenshaw(v, cd) for v in x])
    G = np.array([clenshaw(v, cg) for v in x])
    e1 = float(np.max(np.abs(F / O.F(x) - 1)))
    e2 = float(np.max(np.abs(dF / O.dF(x) - 1)))
    e3 = float(np.max(np.abs(G / O.G0(x) - 1)))
    assert e1 < 2e-15 and e2 < 2e-15 and e3 < 2e-15, (e1, e2, e3)


def test_chebyshev_tail_is_below_rounding(table):
    for c in table:
        assert np.all(np.abs(c[:, -1]) <= 1e-17 * np.abs(c).max(axis=1))
