"""Pins of the oracle's bond-order (Sec. 4.1) and common-neighbour (Sec. 4.2)
analyses: the paper's Tab. Q4Q6 and printed hcp signature, textbook closed
forms of Q_l, the addition theorem, rotation invariance, and hand-built graphs
for the largest-cluster count."""
import math

import numpy as np
import pytest

import mdinputs
from conftest import read_golden
from oracle import boa, cna

D = 2.0 ** (1.0 / 6.0)  # nearest-neighbour distance of the structure workloads
RCNA = 1.2684 * D       # between the first/second shells of fcc/hcp and the 2nd/3rd of bcc


def _lattice(kind):
    if kind == "fcc":
        return mdinputs.fcc_cells((4, 4, 4), D * math.sqrt(2.0))
    if kind == "hcp":
        return mdinputs.hcp_cells((5, 3, 3), D)
    if kind == "bcc":
        a = (2.0 * D ** 3 / math.sqrt(2.0)) ** (1.0 / 3.0)
        return mdinputs.bcc_cells((5, 5, 5), a)
    raise ValueError(kind)


# ---------------------------------------------------------------- BOA
@pytest.mark.parametrize("row", read_golden("q4q6_paper_table.txt"), ids=lambda r: r[0])
def test_q_perfect_lattices_match_paper_table(row):
    kind, nnb, q4, q5, q6 = row[0], int(row[1]), float(row[2]), float(row[3]), float(row[4])
    pos, box = _lattice(kind)
    res = boa.bond_order(pos, box, RCNA, ls=(4, 5, 6))
    assert np.all(res["nu"] == nnb)
    for l, want in ((4, q4), (5, q5), (6, q6)):
        # printed to three decimals
        assert np.all(np.abs(res[l] - want) <= 5e-4 + 1e-12), (kind, l, res[l][:3])
        assert np.ptp(res[l]) < 1e-12  # every atom of a perfect lattice is equivalent


def test_q_closed_forms():
    # simple cubic (6 neighbours): Q4 = sqrt(7/12), Q6 = sqrt(1/8)
    sc = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    assert boa.q_from_directions(sc, 4) == pytest.approx(math.sqrt(7.0 / 12.0), abs=1e-13)
    assert boa.q_from_directions(sc, 6) == pytest.approx(math.sqrt(1.0 / 8.0), abs=1e-13)
    # fcc: Q4 = sqrt(7/192)
    fcc = [np.array(v, float) for v in
           [(1, 1, 0), (1, -1, 0), (-1, 1, 0), (-1, -1, 0), (1, 0, 1), (1, 0, -1),
            (-1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, 1, -1), (0, -1, 1), (0, -1, -1)]]
    assert boa.q_from_directions(fcc, 4) == pytest.approx(math.sqrt(7.0 / 192.0), abs=1e-13)
    # bcc first shell only (8 neighbours): Q4 = sqrt(7/27)
    bcc8 = [np.array((sx, sy, sz), float) for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)]
    assert boa.q_from_directions(bcc8, 4) == pytest.approx(math.sqrt(7.0 / 27.0), abs=1e-13)


def test_q_addition_theorem_cases():
    r = mdinputs.rng(3)
    u = r.standard_normal(3)
    for l in range(0, 9):
        # one neighbour: sum_m |Y_lm|^2 = (2l+1)/(4 pi)  =>  Q_l = 1
        assert boa.q_from_directions([u], l) == pytest.approx(1.0, abs=1e-12)
        # an antipodal pair: Y_lm(-u) = (-1)^l Y_lm(u)
        want = 1.0 if l % 2 == 0 else 0.0
        assert boa.q_from_directions([u, -u], l) == pytest.approx(want, abs=1e-12)


def test_q_rotation_invariant():
    r = mdinputs.rng(8)
    v = r.standard_normal((11, 3))
    R = mdinputs.random_rotation(r)
    for l in (4, 5, 6):
        assert boa.q_from_directions(v @ R.T, l) == pytest.approx(boa.q_from_directions(v, l), abs=1e-12)


def test_q_isolated_atom_is_zero():
    pos = np.array([[1.0, 1.0, 1.0], [5.0, 5.0, 5.0]])
    res = boa.bond_order(pos, np.array([10.0, 10.0, 10.0]), 1.5)
    assert np.all(res["nu"] == 0) and np.all(res[4] == 0) and np.all(res[6] == 0)


# ---------------------------------------------------------------- CNA
@pytest.mark.parametrize(
    "edges,want",
    [
        ([], 0),
        ([(0, 1)], 1),
        ([(0, 1), (2, 3)], 1),             # fcc-like: two disjoint bonds
        ([(0, 1), (1, 2)], 2),             # a path of two bonds
        ([(0, 2), (1, 2)], 2),             # shared larger end
        ([(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (0, 5)], 6),  # hexagon
        ([(0, 1), (1, 2), (0, 2), (5, 7)], 3),
        ([(0, 1), (2, 3), (3, 4), (4, 2), (2, 5)], 4),
    ],
)
def test_max_cluster_hand_graphs(edges, want):
    assert cna.max_cluster_size(edges) == want


def test_cna_fcc_signature():
    pos, box = _lattice("fcc")
    sigs, labels = cna.cna(pos, box, RCNA, atoms=range(0, pos.shape[0], 17))
    for s in sigs.values():
        assert s == [(4, 2, 1)] * 12
    assert set(labels.values()) == {cna.FCC}


def test_cna_hcp_signature_matches_paper():
    want = []
    for n_cn, n_b, n_lcb, count in read_golden("cna_hcp_signature.txt"):
        want += [(int(n_cn), int(n_b), int(n_lcb))] * int(count)
    pos, box = _lattice("hcp")
    sigs, labels = cna.cna(pos, box, RCNA, atoms=range(0, pos.shape[0], 13))
    for s in sigs.values():
        assert s == sorted(want)
    assert set(labels.values()) == {cna.HCP}


def test_cna_bcc_signature():
    pos, box = _lattice("bcc")
    sigs, labels = cna.cna(pos, box, RCNA, atoms=range(0, pos.shape[0], 11))
    for s in sigs.values():
        assert s == sorted([(4, 4, 4)] * 6 + [(6, 6, 6)] * 8)
    assert set(labels.values()) == {cna.BCC}


def test_cna_sampled_equals_full():
    pc = mdinputs.polycrystal(3000, 4, seed=7)
    atoms = list(range(0, pc["pos"].shape[0], 97))
    full_s, full_l = cna.cna(pc["pos"], pc["box"], RCNA, atoms=atoms)
    samp_s, samp_l = cna.cna_sampled(pc["pos"], pc["box"], RCNA, atoms)
    assert full_s == samp_s and full_l == samp_l
    # a jittered polycrystal still has crystalline atoms of several kinds
    assert len(set(full_l.values())) >= 2
