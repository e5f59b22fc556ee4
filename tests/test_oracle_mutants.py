"""Planted mistakes in the oracle are caught by its pins.

Each case copies oracle.c, plants one plausible mistake by a textual edit,
compiles the copy with gcc into a temporary library, points the oracle
binding at it and runs the pin that must fail.  Nothing here touches the
GPU or the committed oracle library.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle as pins

MUTANTS = [
    # name, text in oracle.c, planted replacement, pins that must fail (name, args)
    ("reversed tie order", "    return a.id < b.id;\n}", "    return a.id > b.id;\n}",
     [("test_knn_matches_numpy_bruteforce", ("u8",))]),
    ("budget one short", "                if (t == T) break;", "                if (t + 1 >= T) break;",
     [("test_search_matches_literal_single_queue", (1,))]),
    ("eviction without comparison", "    if (key_less(k, s->e[m])) s->e[m] = k;", "    s->e[m] = k;",
     [("test_bounded_queue_matches_literal_eviction", (1,))]),
    ("wrong multi-sequence children", "    for (int b = last; b < m->P; b++) {", "    for (int b = 0; b < m->P; b++) {",
     [("test_mseq_equals_sort_of_all_tuples", (3, 4))]),
    ("k-means rounding dropped", "int64_t v = (2 * isum[(int64_t)j * ds + e] + cnt[j]) / (2 * cnt[j]);",
     "int64_t v = isum[(int64_t)j * ds + e] / cnt[j];", [("test_kmeans_replay_last_update", ())]),
    ("bridge list order by id only", "    return key_cmp_qsort(&a->k, &b->k);",
     "    return a->k.id < b->k.id ? -1 : (a->k.id > b->k.id);",
     [("test_bridge_graph_top_t_top_b_bruteforce", (3, 2))]),
    ("bf16 ties away from even", "return ((toward >> 16) & 1u) ? (double)fa : (double)ft;",
     "return ((toward >> 16) & 1u) ? (double)ft : (double)fa;",
     [("test_bf16_rounding_matches_library_conversion", ())]),
    ("no re-rank on float rows", "                Rs.e[i].d = sqdist_rows(q, 0, X, Rs.e[i].id, d, 0, d, dtype);",
     "                Rs.e[i].d = Rs.e[i].d;", [("test_bf16_search_is_exact_search_on_rounded_rows_then_rerank", (3,))]),
    ("only the first seed measured", "        int64_t alen = use_bridges ? 0 : nseeds;",
     "        int64_t alen = use_bridges ? 0 : (nseeds > 1 ? 1 : nseeds);",
     [("test_seeded_graph_search_matches_literal", (2,))]),
    ("ADC residual added, not subtracted",
     "const double t = (double)q[j] - (double)centres[(int64_t)l * d + j] - (double)r[e];",
     "const double t = (double)q[j] - (double)centres[(int64_t)l * d + j] + (double)r[e];",
     [("test_ivf_adc_hand_example", ([0, 1, 2], 5, 5, [2, 5, 4, 9, 7], [1, 9.25, 126, 126, 434.25], 5)),
      ("test_ivf_adc_with_exact_codes_is_exact_knn", (10_000,))]),
    ("candidate list cut only at a list's end",
     "for (uint32_t pos = list_off[l]; pos < list_off[l + 1] && c < L; pos++) {",
     "for (uint32_t pos = list_off[l]; pos < list_off[l + 1]; pos++) {",
     [("test_ivf_adc_hand_example", ([1, 0], 2, 3, [2, 7, -1], [1, 434.25, np.inf], 2)),
      ("test_ivf_adc_with_exact_codes_is_exact_knn", (37,))]),
    ("ADC ties to the larger id", "    return (x->id > y->id) - (x->id < y->id);",
     "    return (x->id < y->id) - (x->id > y->id);",
     [("test_ivf_adc_hand_example", ([0, 1, 2], 5, 5, [2, 5, 4, 9, 7], [1, 9.25, 126, 126, 434.25], 5))]),
    ("residual codes tie to the larger codeword", "                if (j == 0 || s < bd) {",
     "                if (j == 0 || s <= bd) {", [("test_pq_encode_matches_bruteforce_argmin", ())]),
]


@pytest.mark.parametrize("name,old,new,must_fail", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, monkeypatch, name, old, new, must_fail):
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site of '{name}' not found once"
    path = tmp_path / "oracle_mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "liboracle_mutant.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-w", "-shared", "-fPIC", str(path), "-o", so, "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle.load(so))
    for pin, args in must_fail:
        with pytest.raises(AssertionError):
            getattr(pins, pin)(*args)


def test_unmutated_copy_passes_the_same_pins(tmp_path, monkeypatch):
    """The harness itself: a copy compiled the same way passes every pin used above."""
    so = str(tmp_path / "liboracle_copy.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-w", "-shared", "-fPIC", oracle.SRC, "-o", so, "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle.load(so))
    for _, _, _, must_fail in MUTANTS:
        for pin, args in must_fail:
            getattr(pins, pin)(*args)
    assert os.path.exists(so)
