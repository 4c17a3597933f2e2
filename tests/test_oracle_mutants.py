"""Mutation tests of the oracle's pins (CPU only).

The oracle source holds a few planted mistakes behind ORC_PLANT (off in the
normal build). Each one is built into its own library here and the pins
named for it are run against that build in a child process: every planted
mistake must make at least one of them fail, while the normal build passes
them (tests/test_oracle_pins.py).
"""
import os
import subprocess
import sys

import pytest

from oracle import build_oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# planted mistake -> pins that must catch it
PLANTS = {
    1: ("dropped opening inner bonded kick of RESPA",
        ["test_respa_inner_loop_is_baoab_on_bonded_water"]),
    2: ("RESPA inner kicks of the outer length",
        ["test_respa_inner_loop_is_baoab_on_bonded_water", "test_jump_respa_samples_the_bond_length_law"]),
    3: ("stale bonded forces inside the RESPA inner loop",
        ["test_respa_inner_loop_is_baoab_on_bonded_water"]),
    4: ("pair histogram bins rounded to the nearest edge",
        ["test_rdf_counts_on_rock_salt_lattice"]),
    5: ("BOUNCE chain without the Coulomb gradient",
        ["test_bounce_j_step_mean_kick_equals_whole_long_force"]),
    6: ("JUMP with Ewald: reciprocal forces left out of the C' acceleration",
        ["test_jump_with_ewald_and_no_long_pairs_is_baoab"]),
    7: ("Ewald sum without the excluded-pair correction",
        ["test_ewald_sum_independent_of_alpha"]),
    8: ("SPME influence function without the B-spline correction",
        ["test_spme_converges_to_the_ewald_sum"]),
    9: ("SPME y force from the B-spline values instead of their derivative",
        ["test_spme_forces_are_minus_energy_gradient", "test_spme_converges_to_the_ewald_sum"]),
    10: ("LJ in the C step jumping on the Coulomb gradient only",
         ["test_c_step_with_lj_in_c_mean_kick_equals_whole_long_force"]),
}


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_mistake_is_caught(plant, tmp_path):
    what, pins = PLANTS[plant]
    lib = build_oracle.build(out=str(tmp_path / f"liboracle_plant{plant}.so"), plant=plant)
    env = dict(os.environ, JUMPMD_ORACLE_LIBRARY=lib)
    caught = []
    for pin in pins:
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            f"tests/test_oracle_pins.py::{pin}"], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=600)
        caught.append(r.returncode != 0)
    assert any(caught), f"planted mistake {plant} ({what}) passed every pin: {pins}"
    # the pins named first are the ones meant for it: all of them must fail
    assert all(caught), f"planted mistake {plant} ({what}) slipped past {[p for p, c in zip(pins, caught) if not c]}"
