"""Host checks of the column FFTs' stage schedule (no GPU).

The column FFT kernels (paper_1808_06736_amd/csrc/kernels_fft.hip) take, per
length L, a list of radices and a block width W (16 or 32 columns).  These tests
read that table from the source and check, on the CPU:
* the radices multiply to L and come in the stated order (4s, at most one 2,
  then 3s, then 5s);
* every stage's butterflies split evenly over the 256 / W threads of a column,
  and the last stage's sub-transform length is a multiple of that count (what
  the kernel's static checks require);
* W = 16 exactly where L is a multiple of 64;
* the lengths the host accepts (fft_cols_supported) are the table's;
* a numpy emulation of the self-sorting (Stockham) schedule with these
  radices, with the kernel's index formulas, equals numpy's FFT for both signs.
The GPU kernels themselves are checked end to end by the parity tests.
"""
import pathlib
import re

import numpy as np
import pytest

SRC = pathlib.Path(__file__).resolve().parents[1] / "paper_1808_06736_amd" / "csrc" / "kernels_fft.hip"


def _table():
    text = SRC.read_text()
    rows = re.findall(r"^\s*ESN_COLS\((\d+),\s*(\d+),\s*([\d,\s]+)\)\s*$", text, re.M)
    out = {}
    for L, W, rs in rows:
        out[int(L)] = (int(W), [int(r) for r in rs.split(",")])
    return out


def _supported():
    text = SRC.read_text()
    body = text[text.index("bool fft_cols_supported"):]
    body = body[:body.index("default:")]
    return sorted(int(v) for v in re.findall(r"case (\d+):", body))


TABLE = _table()


def test_table_is_present_and_matches_the_host_check():
    assert len(TABLE) >= 10
    assert sorted(TABLE) == _supported()


@pytest.mark.parametrize("L", sorted(TABLE))
def test_stage_rules(L):
    W, rs = TABLE[L]
    assert int(np.prod(rs)) == L
    order = {4: 0, 2: 1, 3: 2, 5: 3}
    assert [order[r] for r in rs] == sorted(order[r] for r in rs)
    assert rs.count(2) <= 1
    G = 256 // W
    assert W == (16 if L % 64 == 0 else 32)
    LS = 1
    for i, R in enumerate(rs):
        assert (L // R) % G == 0, (L, R, G)
        if i == len(rs) - 1:
            assert LS % G == 0 and LS * R == L
        LS *= R


def _stockham(x, radices, sgn):
    """The kernel's schedule: stage with sub-length LS and radix R combines, for
    j = q LS + k, the points q LS + k + m L/R twiddled by w^(k m L/(R LS)) into
    q R LS + k + r LS; w = exp(sgn 2 pi i / L)."""
    L = len(x)
    tw = np.exp(sgn * 2j * np.pi * np.arange(L) / L)
    LS = 1
    x = x.astype(np.complex128)
    for R in radices:
        y = np.empty_like(x)
        j = np.arange(L // R)
        k, q = j % LS, j // LS
        a = np.stack([x[q * LS + k + m * (L // R)] * tw[k * m * (L // (R * LS))] for m in range(R)])
        dft = np.exp(sgn * 2j * np.pi * np.outer(np.arange(R), np.arange(R)) / R)
        out = dft.T @ a   # out[r] = sum_m a[m] exp(sgn 2 pi i m r / R)
        for r in range(R):
            y[q * R * LS + k + r * LS] = out[r]
        x = y
        LS *= R
    return x


@pytest.mark.parametrize("L", sorted(TABLE))
@pytest.mark.parametrize("sgn", [-1, 1])
def test_schedule_is_the_dft(L, sgn):
    rng = np.random.default_rng(L)
    x = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    got = _stockham(x, TABLE[L][1], sgn)
    ref = np.fft.fft(x) if sgn < 0 else np.fft.ifft(x) * L
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
