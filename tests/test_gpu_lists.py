"""Interaction lists (Algorithm 1) covered exactly once.

For every layer, each ordered pair of its points (i, j), i = j included, must reach the
free-space sum exactly once: either through a P2P entry of i's leaf whose source range
holds j, or through one M2L entry between an ancestor-or-self of j's leaf and an
ancestor-or-self of i's leaf.  For every reaction component (target tree, source tree)
each pair of a target-tree point and a source-tree point is covered exactly once the same
way.  Equivalently, the pair counts of the P2P lists and of the pairs the M2L chains reach
sum to sum_l N_l^2 (free) and sum over tree pairs of N_t N_s (reaction), with no pair
counted twice.  Checked by dense coverage counts on small plans: uniform, clustered,
six regions, and deep adaptive trees."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _coverage(plan, w):
    st = plan.stats()
    nt = st["n_trees"]
    sizes, layers, sides = [], [], []
    for t in range(nt):
        lay, side, keys, perm = plan.tree(t)
        sizes.append(len(keys))
        layers.append(lay)
        sides.append(side)
    off = np.concatenate([[0], np.cumsum(sizes)])
    boxes = plan.lists(0)
    m2l = plan.lists(1)
    pf = plan.lists(2)
    pr = plan.lists(3)
    start, count = boxes[:, 0].astype(np.int64), boxes[:, 1].astype(np.int64)
    btree = np.searchsorted(off, start, side="right") - 1
    # every box lies inside its tree
    assert np.all(start + count <= off[btree + 1])
    L = len(w["d"])
    free_tree = [t for t in range(nt) if sides[t] == (1 if layers[t] <= L - 1 else 2)]
    cov_f = {t: np.zeros((sizes[t], sizes[t]), np.int16) for t in free_tree}
    cov_r = {(a, b): np.zeros((sizes[a], sizes[b]), np.int16) for a in range(nt) for b in range(nt)}

    def add(cov, tt, ts, t0, tn, s0, sn):
        cov[tt, ts][t0 - off[tt]:t0 - off[tt] + tn, s0 - off[ts]:s0 - off[ts] + sn] += 1

    m2l_free = m2l_reac = 0
    for tb, sb, isfree in m2l:
        tt, ts = btree[tb], btree[sb]
        if isfree:
            assert tt == ts and tt in cov_f
            cov_f[tt][start[tb] - off[tt]:start[tb] - off[tt] + count[tb],
                      start[sb] - off[ts]:start[sb] - off[ts] + count[sb]] += 1
            m2l_free += 1
        else:
            add(cov_r, tt, ts, start[tb], count[tb], start[sb], count[sb])
            m2l_reac += 1
    assert (m2l_free, m2l_reac) == (st["m2l_free_pairs"], st["m2l_reaction_pairs"])
    p2p_pairs = 0
    for lb, s0, sn in pf:
        tt = btree[lb]
        ts = np.searchsorted(off, s0, side="right") - 1
        assert tt == ts and s0 + sn <= off[ts + 1]
        cov_f[tt][start[lb] - off[tt]:start[lb] - off[tt] + count[lb], s0 - off[ts]:s0 - off[ts] + sn] += 1
        p2p_pairs += int(count[lb]) * int(sn)
    rp_pairs = 0
    for lb, s0, sn in pr:
        tt = btree[lb]
        ts = np.searchsorted(off, s0, side="right") - 1
        assert s0 + sn <= off[ts + 1]
        add(cov_r, tt, ts, start[lb], count[lb], s0, sn)
        rp_pairs += int(count[lb]) * int(sn)
    return st, sizes, layers, cov_f, cov_r, p2p_pairs, rp_pairs


@pytest.mark.parametrize("case", ["uniform3", "clustered3", "six_regions", "deep"])
def test_each_pair_covered_exactly_once(case):
    from paper_1908_10863_amd import fmmlm, workloads as W
    if case == "uniform3":
        w, cap, mac = W.config(0), 40, 6
    elif case == "clustered3":
        w, cap, mac = W.config(1, n=3000), 16, 4
    elif case == "six_regions":
        w, cap, mac = W.config(4, n=2400), 12, 6
    else:
        w, cap, mac = W.config(2, n=1500), 3, 4
    _say(f"list coverage {case}: N={len(w['x'])} cap={cap} mac={mac}")
    plan = fmmlm.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=4, leaf_cap=cap, mac_d2=mac)
    try:
        st, sizes, layers, cov_f, cov_r, p2p_pairs, rp_pairs = _coverage(plan, w)
    finally:
        plan.close()
    assert st["m2l_free_pairs"] > 0 and st["m2l_reaction_pairs"] > 0
    # free space: one tree per layer, every ordered pair (self included) exactly once
    assert sorted(layers[t] for t in cov_f) == sorted(set(layers))
    for t, c in cov_f.items():
        assert c.min() == 1 and c.max() == 1, (case, t, c.min(), c.max())
    # reaction: every (target tree, source tree) component, every pair exactly once
    for k, c in cov_r.items():
        assert c.min() == 1 and c.max() == 1, (case, k, c.min(), c.max())
    # the pair counts: P2P pairs (self pairs included) + pairs reached through M2L
    n_l = np.bincount(np.asarray(w["layer"]))
    far_f = sum(int(c.size) for c in cov_f.values()) - p2p_pairs
    assert p2p_pairs + far_f == int(np.sum(n_l.astype(np.int64) ** 2))
    assert p2p_pairs == st["p2p_free_pairs"] and rp_pairs == st["p2p_reaction_pairs"]
    _say(f"  free pairs: {p2p_pairs} by P2P, {far_f} by M2L; reaction: {rp_pairs} by P2P")
