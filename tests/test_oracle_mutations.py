"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a copy of the oracle's C source
(a wrong index, a dropped term, a flipped comparison, rounding in the wrong
place), builds the copy into a temporary library and runs a fixed set of the
CPU pins against it.  At least one pin must fail for every mistake; the
unmodified source built the same way must pass them all.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_adjoint as tadj
import test_oracle_bp as tbp
import test_oracle_dt as tdt
import test_oracle_misc as tmisc
import test_oracle_store16 as ts16

ODIR = os.path.dirname(os.path.abspath(oracle.__file__))
SOURCES = ["bp_oracle.c", "bp_oracle_adjoint.c", "bp_oracle_remap.c", "bp_oracle_features.c"]

# (name, file, text in the source, replacement)
MUTATIONS = [
    ("receiver slot not mirrored", "bp_oracle.c", "int slot = q ^ 1;", "int slot = q;"),
    ("truncation dropped", "bp_oracle.c", "for (int f = 0; f < L; ++f) if (cap < out[f]) out[f] = cap;",
     "for (int f = 0; f < L; ++f) (void)cap;"),
    ("excluded message included", "bp_oracle.c", "if (k != q && has_nb(g, x, y, k)) v += MSG(m, g, k, d, y, x);",
     "if (has_nb(g, x, y, k)) v += MSG(m, g, k, d, y, x);"),
    ("backward pass stops before label 0", "bp_oracle.c", "for (int f = L - 2; f >= 0; --f) {",
     "for (int f = L - 2; f > 0; --f) {"),
    ("forward pass step is half lambda", "bp_oracle.c", "double v = out[f - 1] + lambda;",
     "double v = out[f - 1] + 0.5 * lambda;"),
    ("parent copy from the mirrored slot", "bp_oracle.c",
     "store_round(parent[(((long)k * L + d) * Hp + y / 2) * Wp + x / 2], sm);",
     "store_round(parent[(((long)(k ^ 1) * L + d) * Hp + y / 2) * Wp + x / 2], sm);"),
    ("parent copy not rounded", "bp_oracle.c",
     "store_round(parent[(((long)k * L + d) * Hp + y / 2) * Wp + x / 2], sm);",
     "parent[(((long)k * L + d) * Hp + y / 2) * Wp + x / 2];"),
    ("coarsest level rounded", "bp_oracle.c",
     "int sm = (l == levels - 1 && (store_mode == 1 || store_mode == 2)) ? 0 : store_mode;",
     "int sm = store_mode;"),
    ("message rounded before normalisation", "bp_oracle.c",
     "MSG(m, g, slot, d, ny, nx) = store_round(out[d], store_mode);",
     "MSG(m, g, slot, d, ny, nx) = store_round(out[d] + 0.01, store_mode) - 0.01;"),
    ("argmin ties to the highest label", "bp_oracle.c", "if (v < b[best]) best = d;",
     "if (v <= b[best]) best = d;"),
    ("schedule phase flipped", "bp_oracle.c", "for (int x = (y + t) & 1; x < g->W; x += 2)",
     "for (int x = (y + t + 1) & 1; x < g->W; x += 2)"),
    ("pyramid drops the odd column", "bp_oracle.c", "for (int i = 0; i < 2; ++i) {",
     "for (int i = 0; i < 1; ++i) {"),
    ("data term not truncated", "bp_oracle.c", "v = a < trunc ? a : trunc;", "v = a;"),
    ("downsampling rounds down", "bp_oracle.c", "(uint8_t)((sum + (s * s) / 2) / (s * s))",
     "(uint8_t)(sum / (s * s))"),
    ("soft-argmin temperature inverted", "bp_oracle.c", "double w = exp(-(b[d] - b[best]) / temperature);",
     "double w = exp(-(b[d] - b[best]) * temperature);"),
    ("adjoint drops the normaliser", "bp_oracle_adjoint.c", "hb[gmin] -= mb;", "hb[gmin] -= 0.0 * mb;"),
    ("adjoint lambda term without the absolute value", "bp_oracle_adjoint.c",
     "lsum += mb * fabs((double)(d - gB[d]));", "lsum += mb * (double)(d - gB[d]);"),
    ("adjoint tau term uses tau", "bp_oracle_adjoint.c", "tsum += mb * lambda;", "tsum += mb * tau;"),
    ("adjoint forward-pass tie rule flipped", "bp_oracle_adjoint.c", "if (h[f] <= v) {", "if (h[f] < v) {"),
]

PINS = [
    ("dt worked examples", tdt.test_dt_worked_examples),
    ("dt vs brute force", lambda o: tdt.test_dt_equals_bruteforce_integers(o, 7, 2.0)),
    ("dt numpy definition", tdt.test_dt_numpy_definition_random),
    ("chain min-marginals", lambda o: tbp.test_chain_exact_min_marginals(o, "row", 9, 5, 3.0, 2.0)),
    ("checkerboard = synchronous", lambda o: tbp.test_checkerboard_equals_synchronous(o, 7, 5, 2)),
    ("tree dp", lambda o: tbp.test_tree_dp(o, (5, 4))),
    ("two-level plumbing", lambda o: tbp.test_two_level_plumbing(o, 13, 9)),
    ("pyramid sums", tbp.test_pyramid_sum_random),
    ("soft-argmin closed forms", tbp.test_soft_argmin_closed_forms),
    ("cost worked example", tmisc.test_cost_worked_example),
    ("downsample worked example", tmisc.test_downsample_worked_and_constant),
    ("16-bit coarsest level", lambda o: ts16.test_coarsest_level_keeps_full_precision(o, 1)),
    ("16-bit rounding points", lambda o: ts16.test_rounding_points_match_reference(o, 1, 2, 1, (9, 10, 13))),
    ("adjoint vs finite differences", lambda o: tadj.test_adjoint_matches_finite_differences(o, (8, 5, 6), 6)),
    ("adjoint vs autograd with ties",
     lambda o: tadj.test_adjoint_elementwise_autograd_with_ties(o, (8, 5, 6), 6, 2.0, 2.0)),
]


def _build(tmp_path, name, patch):
    src_dir = tmp_path / name
    src_dir.mkdir()
    for s in SOURCES:
        text = open(os.path.join(ODIR, s)).read()
        if patch and patch[0] == s:
            assert text.count(patch[1]) == 1, f"mutation anchor not unique in {s}: {patch[1]}"
            text = text.replace(patch[1], patch[2])
        (src_dir / s).write_text(text)
    lib = str(src_dir / "liboracle_mut.so")
    subprocess.run(["gcc", "-std=c11", "-O1", "-fPIC", "-shared", "-fopenmp", "-o", lib] +
                   [str(src_dir / s) for s in SOURCES] + ["-lm"], check=True, capture_output=True)
    return lib


def _failing_pins(monkeypatch, lib):
    monkeypatch.setattr(oracle, "_LIB_PATH", lib)
    monkeypatch.setattr(oracle, "_lib", None)
    failed = []
    for name, fn in PINS:
        try:
            with np.errstate(all="ignore"):
                fn(oracle)
        except AssertionError:
            failed.append(name)
    return failed


def test_unmodified_source_passes_the_pins(tmp_path, monkeypatch):
    assert _failing_pins(monkeypatch, _build(tmp_path, "clean", None)) == []


@pytest.mark.parametrize("name,file,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, monkeypatch, name, file, old, new):
    failed = _failing_pins(monkeypatch, _build(tmp_path, "mut", (file, old, new)))
    print(f"{name}: caught by {failed}")
    assert failed, f"no pin fails for the planted mistake '{name}'"
