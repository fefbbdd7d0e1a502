"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU),
builds it, and runs the pin suite against it; the suite must fail.
"""
import os
import subprocess
import sys

import pytest

from oracle import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "cfx_oracle.c")

MUTATIONS = {
    "tie_break_largest_row": ("(a == best && gid[i] < gid[p])", "(a == best && gid[i] > gid[p])"),
    "merge_right_child_first": ("for (int64_t i = 0; i < cl; ++i) gid[i] = cand[a * vb + i];",
                                "for (int64_t i = 0; i < cl; ++i) gid[cr + i] = cand[a * vb + i];"),
    "schur_drops_last_term": ("for (int64_t l = 0; l < vb; ++l) {\n                double a = ri[k + l];",
                              "for (int64_t l = 0; l + 1 < vb; ++l) {\n                double a = ri[k + l];"),
    "l21_wrong_sign": ("for (int64_t l = 0; l < j; ++l) s -= ri[l] * A[(k + l) * lda + k + j];",
                       "for (int64_t l = 0; l < j; ++l) s += ri[l] * A[(k + l) * lda + k + j];"),
    "u12_transposed_operand": ("s -= A[(k + j) * lda + k + l] * A[(k + l) * lda + c];",
                               "s -= A[(k + l) * lda + k + j] * A[(k + l) * lda + c];"),
    "swap_trailing_columns_only": ("for (int64_t c = 0; c < n; ++c) { double t = x[c];",
                                   "for (int64_t c = k; c < n; ++c) { double t = x[c];"),
    "leaf_height_unclamped": ("if (h < vb) h = vb;", ";"),
    "ipiv_relative_index": ("ipiv[k + j] = (int32_t)(k + r);", "ipiv[k + j] = (int32_t)(r);"),
    "gepp_no_elimination": ("blk[i * vb + c] -= l * blk[j * vb + c];", "(void)l;"),
    "eta_no_compensation": ("c += te + pe;", "(void)te; (void)pe;"),
    "min_leaf_count_floor": ("Lk = (n - k + min_leaf - 1) / min_leaf;", "Lk = (n - k) / min_leaf;"),
    "min_leaf_ignored": ("if (min_leaf > 0) {", "if (min_leaf < 0) {"),
    "eta_ignores_non_finite": ("if (bad) return NAN;", "(void)bad;"),
    "merge_uses_partial_values": ("gather_rows(W, ldw, row0, gid, cl + cr, vb, blk);",
                                  "gather_rows(W, ldw, row0, gid, cl + cr, vb, blk); "
                                  "for (int64_t q = cl; q < cl + cr; ++q) for (int64_t c = 0; c < vb; ++c) "
                                  "blk[q * vb + c] -= 0.25 * blk[c];"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor for {name} not unique"
    src = tmp_path / "cfx_oracle.c"
    src.write_text(text.replace(old, new))
    lib = B.build(src=str(src), out=str(tmp_path / "libmut.so"))
    env = dict(os.environ, CFX_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch {name}:\n{r.stdout[-2000:]}"
