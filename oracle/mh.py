"""Independence Metropolis-Hastings chain on log-weights, FP64.

Paper, Sec. 1: flow proposals are corrected to exp(-S)/Z by a Metropolis-Hastings
test "with the Jacobian".  The acceptance formula is not written out; the reading
used here is the independence sampler with proposal density q:

    A(phi -> phi') = min(1, exp(w' - w)),   w = log p - log q = -S - log q.

Decisions use host-drawn log u: accept iff log u < w' - w_cur, computed as one
correctly rounded FP64 subtraction and one compare (no exp), so equal inputs give
bit-equal decisions.  The first proposal a chain ever sees is taken as its
initial state (flagged, not counted as an acceptance).  A rejection repeats the
current configuration.

Chain state (carried across calls): has_state, w_cur, idx_cur (global proposal
number of the current configuration), n_acc, n_seen.

Pinned by: log u = -inf accepts everything; constant w accepts everything (0 > log u
for u < 1); a 1-D independence sampler whose stationary law is known (KS test).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class ChainState:
    has_state: bool = False
    w_cur: float = 0.0
    idx_cur: int = -1
    n_acc: int = 0
    n_seen: int = 0


def mh_chain(logw, log_u, state: ChainState | None = None):
    """Run one chain over proposals k = 0..K-1.  Returns (cur_idx[K], accepted[K], state)."""
    st = ChainState() if state is None else ChainState(**vars(state))
    logw = np.asarray(logw, dtype=np.float64)
    log_u = np.asarray(log_u, dtype=np.float64)
    K = logw.shape[0]
    cur = np.empty(K, dtype=np.int64)
    acc = np.zeros(K, dtype=np.uint8)
    for k in range(K):
        g = st.n_seen + k
        if not st.has_state:
            st.has_state, st.w_cur, st.idx_cur = True, float(logw[k]), g
            acc[k] = 1
        else:
            d = float(logw[k]) - st.w_cur
            if float(log_u[k]) < d:
                st.w_cur, st.idx_cur = float(logw[k]), g
                st.n_acc += 1
                acc[k] = 1
        cur[k] = st.idx_cur
    st.n_seen += K
    return cur, acc, st


def acceptance_rate(state: ChainState) -> float:
    """n_acc / (n_seen - 1): the seeding proposal is not a decision."""
    return state.n_acc / max(state.n_seen - 1, 1)
