"""The library's defaults and the generators of the scenes that stand in for the
paper's are pinned to the values the paper prints (tests/golden/
paper_printed_values.json, each value with its passage)."""
import json
import os

import numpy as np

from paper_2609_02675_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_augmented_lagrangian_constants():
    al = _golden()["augmented_lagrangian"]
    sc = S.mass_ratio_chain(augmented=True)
    assert (sc.al_beta, sc.al_alpha, sc.al_gamma) == (al["beta"], al["alpha"], al["gamma"])
    aug = sc.bond_type == S.BOND_AUGMENTED
    assert aug.all() and np.all(sc.kappa[aug] == al["kappa_start"])
    # a plain scene description carries the same constants by default
    plain = S.chain8()
    assert (plain.al_beta, plain.al_alpha, plain.al_gamma) == (al["beta"], al["alpha"], al["gamma"])


def test_spring_net_shape():
    g = _golden()["spring_net"]
    net = S.spring_net()
    assert net.n_bodies == g["grid"] ** 2
    assert net.n_bonds == g["springs"]
    deg = np.bincount(np.concatenate([net.bond_i, net.bond_j]), minlength=net.n_bodies).reshape(g["grid"], g["grid"])
    assert np.all(deg[1:-1, 1:-1] == g["neighbours_per_interior_box"])


def test_mass_ratio_chain_matches_its_table_row():
    row = _golden()["table2_mass_ratio_chain"]
    for aug in (True, False):
        sc = S.mass_ratio_chain(augmented=aug)
        assert (sc.n_bodies, sc.n_bonds, sc.iters) == (row["bodies"], row["joints"], row["iterations"])


def test_block_pile_matches_its_table_row():
    """The stand-in keeps the 50^3 blocks and the iteration count; the impacting
    ball of the paper's scene is left out (125,000 of its 125,001 bodies)."""
    row = _golden()["table2_block_pile"]
    sc = S.block_pile()
    assert sc.n_bodies == row["blocks_per_side"] ** 3 == row["bodies"] - 1
    assert sc.n_bonds == row["joints"] and sc.iters == row["iterations"]
