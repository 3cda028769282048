"""Planted mistakes in the oracle must fail its pins.

Each mutant is a copy of pedsim_oracle.c with one plausible slip (a swapped
operand, a wrong sign, a dropped term, a reversed comparison), compiled on
the CPU into a temporary library; the pin suite is then run against it and
must fail. This shows the pins constrain every part of the oracle.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pedsim_oracle.c")

MUTANTS = {
    "philox_high_halves_swapped": ("x0 = hi1 ^ x1 ^ k0;", "x0 = hi0 ^ x1 ^ k0;"),
    "philox_key_bumped_before_first_round": ("if (round > 0) {", "if (round >= 0) {"),
    "lem_side_order_ignored": ("(r2 & 1u) ? plus_first : minus_first;\n  int ranked[7];",
                               "(r2 & 0u) ? plus_first : minus_first;\n  int ranked[7];"),
    "lem_threshold_index_dropped": ("if (r1 >= lem_threshold[i]) index += 1;",
                                    "if (r1 >= lem_threshold[0]) index += 1;", 0),
    "aco_weights_swapped": ("eta[0] = eta[1] = heuristic_weight(D2_DIAGONAL, p->beta);",
                            "eta[0] = eta[1] = heuristic_weight(D2_LATERAL, p->beta);"),
    "aco_uses_r2": ("u = (float)(r1 >> 8) * 0x1p-24f;", "u = (float)(r2 >> 8) * 0x1p-24f;", 0),
    "aco_alpha_ignored": ("if (avail[i]) {\n      float power = 1.0f;\n      int a;\n      if (alpha > 0) {\n"
                          "        power = tau[i];\n        for (a = 1; a < alpha; ++a)",
                          "if (avail[i]) {\n      float power = 1.0f;\n      int a;\n      if (alpha > 0) {\n"
                          "        power = tau[i];\n        for (a = 1; a < 1; ++a)"),
    "deposit_before_evaporation": ("float va = keep * tau_a[c];",
                                   "float va = keep * (tau_a[c] + (code[c] == O_A ? p->dtau : 0.0f));", 0),
    "winner_highest_ticket": ("w[0] < best_ticket || (w[0] == best_ticket && k < best_k)",
                              "w[0] > best_ticket || (w[0] == best_ticket && k < best_k)"),
    "source_id_not_cleared": ("new_id[n] = 0;", "(void)0;"),
    "diagonal_sign_flipped": ("case O_REQ_FDP: *tx = x + d; *ty = y + 1; break;",
                              "case O_REQ_FDP: *tx = x + d; *ty = y - 1; break;"),
    "b_heads_plus_x": ("return group == O_A ? 1 : -1;", "return 1;"),
    "forward_first_dropped": ("if (free_cell(p, code, x + d, y)) return O_REQ_F;", ""),
    "other_groups_pheromone": ("(g == O_A) ? tau_a : tau_b", "(g == O_A) ? tau_b : tau_a", 0),
    "tour_diagonal_counts_one": ("(best_dx != 0 && best_dy != 0) ? diagonal_step : 1.0f", "1.0f"),
    "tour_deposit_on_occupied": ("if (entered[c] == O_A) evaporated_a",
                                 "if (code[c] == O_A) evaporated_a"),
    "tour_deposit_not_divided": ("evaporated_a + p->dtau / tour[id[c] - 1u]",
                                 "evaporated_a + p->dtau"),
    "tour_entered_cell_not_evaporated": (
        "float evaporated_a = keep * tau_a[c];",
        "float evaporated_a = entered[c] == O_A ? tau_a[c] : keep * tau_a[c];"),
    "tour_b_deposit_on_a_plane": (
        "if (entered[c] == O_B) evaporated_b = evaporated_b + p->dtau / tour[id[c] - 1u];",
        "if (entered[c] == O_B) evaporated_a = evaporated_a + p->dtau / tour[id[c] - 1u];"),
    "tour_group_of_target_not_mover": ("entered[c] = code[n];", "entered[c] = code[c];"),
    "nb8_backward_is_forward": ("case O_REQ_B: *tx = x - d; break;", "case O_REQ_B: *tx = x + d; break;"),
    "nb8_back_diagonal_sign": ("case O_REQ_BDP: *tx = x - d; *ty = y + 1; break;",
                               "case O_REQ_BDP: *tx = x - d; *ty = y - 1; break;"),
    "nb8_back_weights_swapped": ("eta[4] = heuristic_weight(D2_BACKWARD, p->beta);",
                                 "eta[4] = heuristic_weight(D2_BACK_DIAGONAL, p->beta);"),
    "nb8_back_pair_order_fixed": ("O_REQ_B, O_REQ_BDP, O_REQ_BDM};", "O_REQ_B, O_REQ_BDM, O_REQ_BDP};"),
    "nb8_three_thresholds_only": ("for (i = 0; i < sides - 1; ++i)", "for (i = 0; i < 3; ++i)"),
    "crossing_edge_strict": ("if (x >= p->W - p->cross_b) crossed_a += 1;",
                             "if (x > p->W - p->cross_b) crossed_a += 1;"),
    "crossing_bands_swapped": ("if (x >= p->W - p->cross_b) crossed_a += 1;",
                               "if (x >= p->W - p->cross_a) crossed_a += 1;"),
    "crossing_b_edge_inclusive": ("if (x < p->cross_a) crossed_b += 1;",
                                  "if (x <= p->cross_a) crossed_b += 1;"),
    "crossing_b_band_swapped": ("if (x < p->cross_a) crossed_b += 1;",
                                "if (x < p->cross_b) crossed_b += 1;"),
    # larger scanning and moving ranges
    "range_scan_limited_to_move": ("f[r] = free_run(p, code, x, y, ux[r], uy[r], S);",
                                   "f[r] = free_run(p, code, x, y, ux[r], uy[r], M);"),
    "range_move_not_capped": ("len[c] = (uint8_t)(f[choice] < M ? f[choice] : M);",
                              "len[c] = (uint8_t)(f[choice]);"),
    "range_score_reversed": ("if ((int64_t)f[q] * f[q] * d2[r] < (int64_t)f[r] * f[r] * d2[q]) {",
                             "if ((int64_t)f[q] * f[q] * d2[r] > (int64_t)f[r] * f[r] * d2[q]) {"),
    "range_score_ignores_run": ("if ((int64_t)f[q] * f[q] * d2[r] < (int64_t)f[r] * f[r] * d2[q]) {",
                                "if (d2[r] < d2[q]) {"),
    "range_reference_two_ahead": ("int64_t dx = (int64_t)(M + 1) - (int64_t)a * k;",
                                  "int64_t dx = (int64_t)2 - (int64_t)a * k;"),
    "range_weight_ignores_visibility": (
        "return (float)(pow((double)f / (double)S, (double)beta) * pow(d2, -0.5 * (double)beta));",
        "return (float)(pow(d2, -0.5 * (double)beta));"),
    "range_tau_next_to_agent": ("tau[r] = plane[(size_t)(y + k * uy[r]) * W + (size_t)(x + k * ux[r])];",
                                "tau[r] = plane[(size_t)(y + uy[r]) * W + (size_t)(x + ux[r])];"),
    "range_forward_not_first": ("      if (f[0] >= 1) {\n        choice = 0; /* forward first */",
                                "      if (0) {\n        choice = 0; /* forward first */"),
    "range_gather_radius_one": ("for (dy = -M; dy <= M; ++dy)\n        for (dx = -M; dx <= M; ++dx) {",
                                "for (dy = -1; dy <= 1; ++dy)\n        for (dx = -1; dx <= 1; ++dx) {"),
    "range_side_order_ignored": ("(r2 & 1u) ? plus_first : minus_first;\n  int ranked[4];",
                                 "(r2 & 0u) ? plus_first : minus_first;\n  int ranked[4];"),
    "range_aco_alpha_ignored": ("if (f[i] >= 1) {\n      float power = 1.0f;\n      int a;\n      if (alpha > 0) {\n"
                                "        power = tau[i];\n        for (a = 1; a < alpha; ++a)",
                                "if (f[i] >= 1) {\n      float power = 1.0f;\n      int a;\n      if (alpha > 0) {\n"
                                "        power = tau[i];\n        for (a = 1; a < 1; ++a)"),
    "range_deposit_before_evaporation": ("float va = keep * tau_a[c];",
                                         "float va = keep * (tau_a[c] + (code[c] == O_A ? p->dtau : 0.0f));", 1),
    "range_aco_uses_r2": ("u = (float)(r1 >> 8) * 0x1p-24f;", "u = (float)(r2 >> 8) * 0x1p-24f;", 1),
    "range_threshold_index_dropped": ("if (r1 >= lem_threshold[i]) index += 1;",
                                      "if (r1 >= lem_threshold[0]) index += 1;", 1),
    "range_other_groups_pheromone": ("(g == O_A) ? tau_a : tau_b", "(g == O_A) ? tau_b : tau_a", 1),
    "range_winner_highest_ticket": ("if (!have || w[0] < best_ticket || (w[0] == best_ticket && kk < best_k)) {",
                                    "if (!have || w[0] > best_ticket || (w[0] == best_ticket && kk < best_k)) {"),
}


def _run_mutant(name):
    """Compile the mutant and run the pins against it; returns the pin run's
    exit status (0 = the mutant passed every pin)."""
    old, new = MUTANTS[name][:2]
    nth = MUTANTS[name][2] if len(MUTANTS[name]) > 2 else None
    with open(SRC) as f:
        src = f.read()
    if nth is None:
        assert src.count(old) == 1, f"mutation anchor for {name} not unique"
        nth = 0
    # the base model and the range model share some lines: nth picks which copy
    assert src.count(old) > nth, f"mutation anchor for {name} missing"
    at = -1
    for _ in range(nth + 1):
        at = src.index(old, at + 1)
    pins = [os.path.join(ROOT, "tests", "test_oracle_pins.py"),
            os.path.join(ROOT, "tests", "test_oracle_range_pins.py")]
    if name.startswith("range_"):  # the range pins first: they stop a range mutant sooner
        pins.reverse()
    with tempfile.TemporaryDirectory() as d:
        msrc = os.path.join(d, "mutant.c")
        mlib = os.path.join(d, "libmutant.so")
        with open(msrc, "w") as f:
            f.write(src[:at] + new + src[at + len(old):])
        subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                        "-o", mlib, msrc, "-lm"], check=True)
        env = dict(os.environ, PEDSIM_ORACLE_LIB=mlib, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *pins],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
        return r.returncode


@pytest.fixture(scope="module")
def mutant_status():
    """Every mutant's pin run, several at a time (each is one CPU-bound
    process), so the suite's wall time stays a few minutes."""
    workers = max(1, min(8, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                         else (os.cpu_count() or 1)))
    with ThreadPoolExecutor(workers) as ex:
        return dict(zip(sorted(MUTANTS), ex.map(_run_mutant, sorted(MUTANTS))))


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name, mutant_status):
    assert mutant_status[name] != 0, f"mutant {name} passed every pin"
