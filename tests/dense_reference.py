"""An independent, vectorised statement of the spatial pooler step used to
pin the oracle (test helper; not the oracle, shares no code with it).

  overlap    raw = X @ M, M[n, c] = number of connected synapses of c on input
             n (integer matrix product), gated at min_overlap (Section 1.1,
             Algorithm 1, boost 1);
  inhibition np.lexsort by (overlap descending, index ascending), keeping
             positive overlaps, first k (Algorithm 2, global form);
  learning   q' = clip(q + inc*x - dec*(1 - x), 0, 256) on the winners' rows,
             in integer 1/256 units (the whitepaper rule the paper defers to).
"""
import numpy as np

from paper_1608_01966_amd import synth


def dense_run(cfg, idx, perm_q, frames, learn=True):
    N, C, S = cfg["input_bits"], cfg["num_columns"], cfg["synapses_per_column"]
    k, m = cfg["winners"], cfg["min_overlap"]
    q = np.array(perm_q, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    X = synth.unpack_bits(np.asarray(frames, dtype=np.uint32), N).astype(np.int64)
    F = X.shape[0]
    ovs = np.zeros((F, C), dtype=np.int64)
    wins = np.full((F, k), -1, dtype=np.int64)
    cols = np.repeat(np.arange(C), S).reshape(C, S)
    for t in range(F):
        conn = q >= cfg["connected_q8"]
        M = np.zeros((N, C), dtype=np.int64)
        np.add.at(M, (idx[conn], cols[conn]), 1)
        raw = X[t] @ M
        ov = np.where(raw >= m, raw, 0)
        order = np.lexsort((np.arange(C), -ov))
        order = order[ov[order] > 0][:k]
        w = np.sort(order)
        wins[t, :w.size] = w
        ovs[t] = ov
        if learn and w.size:
            x = X[t][idx[w]]
            q[w] = np.clip(q[w] + cfg["inc_q8"] * x - cfg["dec_q8"] * (1 - x), 0, 256)
    return ovs, wins, q
