"""Oracle: common-neighbour analysis with literal Python sets (Sec. 4.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Bonds: i and v are bonded iff |r_i - r_v| < rc (min image, strict, the exact
predicate of ``oracle.lj``).  For atom i the paper forms

    E_d(i) = {(i, v) : v bonded to i}                              (Eq. Ei)
    Ebar(i) = {(v, w) : v bonded to i, w bonded to v, w != i}      (Eq. Ei;
              the w != i exclusion is the one Alg. cna_II applies)

and for every bonded pair (i, j)

    C = N(i) & N(j)                         common neighbours
    E = {(v, w) : v, w in C, v < w, bonded} common-neighbour bonds,
        gathered from Ebar(i) with both ends in C, stored ordered v < w
    triplet = (|C|, |E|, maxClustersize(E))  (Alg. cna_III)

maxClustersize follows Alg. max_cluster_size: repeatedly take an edge,
breadth-first traverse from one of its ends, count and remove every edge
met, keep the largest count.

Readings: an edge (v, w) is met from either end (the algorithm's
"(v, w) in E" is read as "incident to v"; with ordered pairs only, two edges
sharing their larger end would split into two clusters, breaking the hcp
signature the paper prints); the third triplet entry counts edges (the
algorithm's count), which the fcc (4,2,1) signature also requires.

Labels (Stukowski's reference signatures, cited by the paper):
    FCC: 12 bonds, all (4,2,1)
    HCP: 12 bonds, six (4,2,1) and six (4,2,2)   (printed in Sec. 4.2)
    BCC: 14 bonds, eight (6,6,6) and six (4,4,4)
    otherwise OTHER
"""
from __future__ import annotations

from collections import Counter

import numpy as np

from .lj import neighbour_pairs, local_subset

OTHER, FCC, HCP, BCC = 0, 1, 2, 3


def neighbour_sets(pos, box, rc: float, rows=None):
    """dict atom -> set of bonded atoms (strict rc, min image)."""
    pos = np.asarray(pos, dtype=np.float64)
    r2 = float(rc) * float(rc)
    pairs = neighbour_pairs(pos, box, r2, rows)
    nb = {}
    keys = range(pos.shape[0]) if rows is None else rows
    for i in keys:
        nb[int(i)] = set()
    for i, j in pairs:
        nb[int(i)].add(int(j))
    return nb


def direct_bonds(nb, i):
    return {(i, v) for v in nb[i]}


def indirect_bonds(nb, i):
    out = set()
    for v in nb[i]:
        for w in nb[v]:
            if w != i:
                out.add((v, w))
    return out


def max_cluster_size(edges) -> int:
    """Alg. max_cluster_size: largest number of edges in one connected component."""
    E = set(edges)
    s_max = 0
    while E:
        s = 0
        v1, _ = next(iter(E))
        queue = [v1]
        while queue:
            v = queue.pop(0)
            P = {e for e in E if v in e}
            for e in P:
                queue.append(e[1] if e[0] == v else e[0])
            s += len(P)
            E -= P
        s_max = max(s, s_max)
    return s_max


def triplet(nb, i, j, ebar_i=None):
    """(n_cn, n_b, n_lcb) of the bonded pair (i, j)."""
    C = {v for (_, v) in direct_bonds(nb, i)} & {v for (_, v) in direct_bonds(nb, j)}
    if ebar_i is None:
        ebar_i = indirect_bonds(nb, i)
    E = set()
    for (v, w) in ebar_i:
        if v in C and w in C:
            if w < v:
                v, w = w, v
            E.add((v, w))
    return (len(C), len(E), max_cluster_size(E))


def atom_signature(nb, i):
    """Sorted list of triplets over the bonds of atom i."""
    eb = indirect_bonds(nb, i)
    return sorted(triplet(nb, i, j, eb) for j in nb[i])


def classify(sig) -> int:
    c = Counter(sig)
    n = len(sig)
    if n == 12 and c[(4, 2, 1)] == 12:
        return FCC
    if n == 12 and c[(4, 2, 1)] == 6 and c[(4, 2, 2)] == 6:
        return HCP
    if n == 14 and c[(6, 6, 6)] == 8 and c[(4, 4, 4)] == 6:
        return BCC
    return OTHER


def cna(pos, box, rc: float, atoms=None):
    """Signatures and labels for ``atoms`` (default all).

    Uses all-pairs neighbour sets of the whole system.  Returns
    (signatures: dict atom -> sorted triplets, labels: dict atom -> int)."""
    nb = neighbour_sets(pos, box, rc)
    atoms = range(len(nb)) if atoms is None else atoms
    sigs, labels = {}, {}
    for i in atoms:
        s = atom_signature(nb, int(i))
        sigs[int(i)] = s
        labels[int(i)] = classify(s)
    return sigs, labels


def cna_sampled(pos, box, rc: float, atoms):
    """Like ``cna`` for a few atoms of a large system: each atom is analysed
    on the atoms within 2 rc (+ margin) of it, which contain every bond its
    triplets read."""
    pos = np.asarray(pos, dtype=np.float64)
    sigs, labels = {}, {}
    for i in atoms:
        sub = local_subset(pos, box, int(i), 2.0 * rc * (1.0 + 1e-9) + 1e-9)
        # neighbour sets on the subset, then mapped back to global ids
        nb_local = neighbour_sets(pos[sub], box, rc)
        gid = {k: int(sub[k]) for k in range(sub.shape[0])}
        nb = {gid[k]: {gid[m] for m in s} for k, s in nb_local.items()}
        s = atom_signature(nb, int(i))
        sigs[int(i)] = s
        labels[int(i)] = classify(s)
    return sigs, labels
