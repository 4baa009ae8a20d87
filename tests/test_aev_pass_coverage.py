"""The AEV parity cases reach every branch of the forward kernel's pass plan.

The forward takes the angular pairs of a centre in passes of 64 slots: a
species-pair block with more than 64 pairs left fills a pass alone,
otherwise the pass holds the rest of that block followed by whole smaller
blocks, each padded to a multiple of 8 slots.  This CPU test replays that
plan on the ragged 16-solute case that the GPU parity test compares with
the oracle feature by feature, and checks that the case contains multi-pass
blocks, blocks of exactly a multiple of 64 pairs, passes that start with
the tail of a large block and then take further blocks, passes of four or
more blocks, and single-pair blocks.
"""
import numpy as np

import synth

SLOTS = 64


def block_sizes(coords, species, i, rc_a, n_species):
    d = np.linalg.norm(coords - coords[i], axis=1)
    d[i] = np.inf
    cnt = np.bincount(species[d < rc_a], minlength=n_species)
    sizes = [cnt[a] * (cnt[a] - 1) // 2 if a == b else cnt[a] * cnt[b]
             for a in range(n_species) for b in range(a, n_species)]
    return [t for t in sizes if t > 0]


def replay(sizes):
    """Passes of one centre as lists of (block, first pair, pairs taken)."""
    passes, q, u = [], 0, 0
    while q < len(sizes):
        if sizes[q] - u > SLOTS:
            passes.append([(q, u, SLOTS)])
            u += SLOTS
            continue
        cur, used, k = [(q, u, sizes[q] - u)], (sizes[q] - u + 7) // 8 * 8, q + 1
        while k < len(sizes) and used + (sizes[k] + 7) // 8 * 8 <= SLOTS:
            cur.append((k, 0, sizes[k]))
            used += (sizes[k] + 7) // 8 * 8
            k += 1
        passes.append(cur)
        q, u = k, 0
    return passes


def test_replay_covers_every_pair_once():
    for sizes in ([1], [64], [65], [128, 3], [7, 9, 1, 30, 64, 200, 8, 8, 8, 8, 8, 8, 8, 8]):
        seen = {}
        for p in replay(sizes):
            assert sum((n + 7) // 8 * 8 for _, _, n in p) <= SLOTS
            for blk, first, n in p:
                for t in range(first, first + n):
                    seen[(blk, t)] = seen.get((blk, t), 0) + 1
        assert sorted(seen) == [(b, t) for b, s in enumerate(sizes) for t in range(s)]
        assert set(seen.values()) == {1}


def test_ragged_parity_case_reaches_every_branch():
    b = synth.ragged_solutes(16, seed=12)
    p = synth.aev_params()
    cov = dict(multi_pass=0, multiple_of_64=0, tail_then_more=0, four_or_more=0, single_pair=0)
    for k in range(b.n_systems):
        a, e = int(b.offsets[k]), int(b.offsets[k + 1])
        x, s = b.coords[a:e].astype(np.float64), b.species[a:e]
        for i in range(e - a):
            sizes = block_sizes(x, s, i, p["rc_ang"], 7)
            cov["multi_pass"] += sum(t > SLOTS for t in sizes)
            cov["multiple_of_64"] += sum(t >= SLOTS and t % SLOTS == 0 for t in sizes)
            cov["single_pair"] += sum(t == 1 for t in sizes)
            for ps in replay(sizes):
                cov["four_or_more"] += len(ps) >= 4
                cov["tail_then_more"] += ps[0][1] > 0 and len(ps) >= 2
    assert all(v > 0 for v in cov.values()), cov
