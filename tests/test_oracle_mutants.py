"""Plant plausible mistakes in copies of the oracle (CPU only) and check that
the pins in test_oracle_pins catch every one of them."""
import ctypes
import os
import subprocess

import pytest

from oracle import oracle as O
from tests import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(O.__file__), "oracle.c")

# (description, original text, mutated text)
MUTANTS = [
    ("sign of an imaginary part in type 1", "row[2 * a1 + 1] += u2r", "row[2 * a1 + 1] -= u2r"),
    ("mode offset for odd N in type 2", "ks[m][a] = a - Ns[m] / 2;", "ks[m][a] = a - (Ns[m] + 1) / 2;"),
    ("transposed coordinate", "phases(jb->x[1][j], jb->isign, n2, jb->k[1], e2);",
     "phases(jb->x[0][j], jb->isign, n2, jb->k[1], e2);"),
    ("dropped last term", "for (int64_t j = jb->j0; j < jb->j1; j++) {",
     "for (int64_t j = jb->j0; j < jb->j1 - (jb->j1 > jb->j0 + 1); j++) {"),
    ("ignored isign", "double th = (double)isign * (double)k[a] * x;", "double th = (double)k[a] * x;"),
    ("conjugated product in type 2", "bi += fr * pi + fi * pr;", "bi += fr * pi - fi * pr;"),
    ("unfinished block left out of a type 2 sum", "jb->out[2 * j] = sr + br;", "jb->out[2 * j] = sr;"),
    ("block sums of type 1 not added", "for (int64_t q = 0; q < 2 * K; q++) acc[q] += blk[q];",
     "for (int64_t q = 0; q < 2 * K; q++) acc[q] = blk[q];"),
]

PINS = [
    (P.test_type1_uniform_grid_is_dft, [((7,), 1), ((6, 5), -1), ((4, 7), 1), ((5, 4, 3), 1),
                                        ((5003,), 1)]),
    (P.test_type2_uniform_grid_is_dft, [((9,), 1), ((6, 5), -1), ((4, 3, 5), -1), ((5003,), -1)]),
    (P.test_adjointness, [(1, (13,), 40), (2, (6, 9), 50), (3, (5, 4, 7), 30)]),
    (P.test_translation_and_period, [(1,), (-1,)]),
    (P.test_type2_single_mode, [()]),
]


def _load_mutant(tmp_path, old, new):
    text = open(SRC).read()
    assert old in text, old
    src = tmp_path / "mut.c"
    src.write_text(text.replace(old, new, 1))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", str(lib), str(src),
                           "-lm", "-lpthread"])
    return str(lib)


@pytest.mark.parametrize("desc,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, monkeypatch, desc, old, new):
    lib = _load_mutant(tmp_path, old, new)
    monkeypatch.setattr(O, "_LIB", lib)
    monkeypatch.setattr(O, "_lib", None)
    caught = 0
    for fn, cases in PINS:
        for args in cases:
            try:
                fn(*args)
            except AssertionError:
                caught += 1
    assert caught > 0, f"no pin caught: {desc}"
