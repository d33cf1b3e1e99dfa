"""The oracle's pins catch plausible mistakes.

Each case compiles a copy of oracle.c with one planted slip (on the CPU, in a
temporary directory) and checks that at least one pin fails on it, while the
unmodified oracle passes the same pins (test_oracle_pins.py).  The slips are
the ones a reader could make when writing the method down: the backward
stage's node means (Sec. 2.2, backward stage), a dropped adjoint term, the
literal single /n_k momentum of an approximated node (eq. 4), the far-field
test without its square, and a wrong running-mean denominator of the node
centre (Sec. 2.2, node statistics).
"""
import importlib.util
import os
import subprocess

import pytest

import test_oracle_pins as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PY = os.path.join(ROOT, "oracle", "oracle.py")

MUTATIONS = {
    "node_mean_beta": ("double mb[3] = {bj[0] / wcount, bj[1] / wcount, bj[2] / wcount};",
                       "double mb[3] = {bj[0], bj[1], bj[2]};"),
    "dropped_alpha_term": ("double cross = dot3(pj, ak) + dot3(pk, aj);",
                           "double cross = dot3(pj, ak);"),
    "literal_single_over_n": ("v[c] += g * k->P[c];", "v[c] += g * k->P[c] / (double)k->n;"),
    "far_test_unsquared": ("int far = dmin2 >= cut * cut;", "int far = dmin2 >= cut;"),
    "centre_denominator": ("nd->C[c] = (nd->C[c] * nold + qj[c]) / (nold + 1.0);",
                           "nd->C[c] = (nd->C[c] * nold + qj[c]) / (nold + 2.0);"),
}

# pins run against each mutant; a mutant must fail at least one of them
PINS = [
    lambda O: P.test_rhs_is_hamiltonian_vector_field(O, 7, 2),
    lambda O: P.test_adjoint_matches_autograd(O),
    lambda O: P.test_bh_exact_on_coincident_far_clusters(O),
    lambda O: P.test_bh_matches_bruteforce(O, 0.5, 3),
    lambda O: P.test_tree_matches_brute_force_cells(O, 3),
]


def _mutant(tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not found once"
    c = tmp_path / f"oracle_{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"liboracle_{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                    "-fPIC", "-shared", "-o", str(so), str(c), "-lm"], check=True)
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{name}", PY)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB = str(so)
    mod.build = lambda force=False: mod._LIB
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(tmp_path, name):
    O = _mutant(tmp_path, name)
    caught = []
    for pin in PINS:
        try:
            pin(O)
        except AssertionError:
            caught.append(pin)
    assert caught, f"no pin fails on the planted mistake {name}"
