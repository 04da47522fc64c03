"""Shared check of the plan pass's ranks against top-k lists (used by the GPU tests)."""
import numpy as np


def check_ranks_against_lists(rank, truth, val, idx):
    """The plan pass's rank of each true partner t (1 + #{j : y_ij > y_it}) against the
    top-k list of the same row.  Entries listed before t have y >= y_t, those with a
    strictly larger FP32 value strictly larger y, so a listed partner at position pos
    has  #{q < pos : val_q > val_pos} <= rank - 1 <= pos  (equal when no FP32 value
    ties; exact exponent ties, e.g. a row splitting its mass evenly, list the lower
    column first but do not count in the rank).  An unlisted partner has y_t <= y of
    the last entry, so rank - 1 >= #{q : val_q > val_last}."""
    k = idx.shape[1]
    rows = np.nonzero(rank > 0)[0]
    for i in rows:
        pos = np.nonzero(idx[i] == truth[i])[0]
        if pos.size:
            q = int(pos[0])
            lo = int(np.count_nonzero(val[i, :q] > val[i, q]))
            assert lo <= rank[i] - 1 <= q, (i, rank[i], q, lo)
        else:
            assert rank[i] - 1 >= int(np.count_nonzero(val[i] > val[i, k - 1])), (i, rank[i])
    return rows
