"""Host-side checks of split features and candidate splits (no GPU)."""
import math

import numpy as np

import paper_2608_01467_amd as fhs
import workloads as w


def test_candidate_splits_cover_eq8_optimum():
    for text in (w.quantum_walk(20, 9).to_text(), w.qaoa_maxcut(8, 2, 3, 4)[0].to_text(),
                 w.amplitude_amplification(3, 2, 4, 5)[0].to_text(),
                 w.random_mixed(6, 40, 11).to_text()):
        p = fhs.Program(text)
        cand = p.candidate_splits()
        assert len(cand) == (p.A + 1) * (p.A + 2) // 2
        assert all(c1 <= c2 <= p.G for c1, c2 in cand)
        best_any = p.partition_cost(*p.choose_partition(fhs.PART_EQ8))[0]
        best_cand = min(p.partition_cost(*c)[0] for c in cand)
        assert best_cand == best_any          # the Eq. (8) optimum lies on the grid


def test_features_match_regions_and_eq8():
    p = fhs.Program(w.quantum_walk(99, 20).to_text())
    for c1, c2 in p.candidate_splits()[::17]:
        f = p.split_features(c1, c2, 8192, 1)
        cost, reg = p.partition_cost(c1, c2)
        assert tuple(int(x) for x in f[:3]) == reg[3:]
        assert abs(f[12] - math.log2(1 + cost)) < 1e-12
        assert f[10] == 13.0 and f[11] == 4.0
        assert abs(f[13] - (13 + reg[3] + reg[4])) < 1e-12
        # suffix work: 2^A histories x the suffix's work per history
        e2 = max(c2, p.L)
        wk = p.work(e2, p.G)
        assert abs(f[7] - math.log2(1 + 2 ** p.A * wk["int_ops"])) < 1e-9
        assert f[15] <= f[14] and f[14] > 0
