"""Pure-Python loop form of flood GaBP for nonsymmetric matrices (test infrastructure only).

Follows the reparametrised message rules of Sec. 2.3 (eq. nonsymmetric_GaBP_rules) term by
term, in the paper's notation, with the flood schedule of Sec. 2.2: every message of
iteration n+1 is computed from messages of iteration n only.

Graph (Sec. 2.3): a directed edge j -> i exists iff A_ij != 0 (i != j). The message it
carries is the pair (Lt_ji, m_ji) = (Lambda~_ji, m_ji).

One iteration of Algorithm 1 (flood form), for every node j:
    m     = b_j + sum_{k in N(j)} m_kj
    Sigma = A_jj + sum_{k in N(j)} Lt_kj A_kj
    x_j   = m / Sigma
and for every edge j -> i:
    Lt_ji <- -A_ij / (Sigma - Lt_ij A_ij)
    m_ji  <- Lt_ji (m - m_ij)
where N(j) are the senders into j and a missing reverse message (A_ji = 0) counts as 0.

Only for small matrices (<= ~10^4 edges).
"""
from __future__ import annotations


def _entries(n, rowptr, col, val):
    a = {}
    for i in range(n):
        for t in range(int(rowptr[i]), int(rowptr[i + 1])):
            v = float(val[t])
            if v != 0.0:
                a[(i, int(col[t]))] = v
    return a


def gabp_loops(n, rowptr, col, val, b, sweeps, Lt=None, m=None, lambda_only=False):
    """Run ``sweeps`` iterations of Algorithm 1 (flood schedule) from the given messages.

    Returns ``(x, Lt, m, Sigma)``: x and Sigma are the read-off of the last iteration (built
    from the messages *before* that iteration's update, as in Algorithm 1), Lt and m the
    messages after ``sweeps`` updates. Messages are dicts keyed (sender, receiver).
    Zero initial messages when Lt/m are None.
    """
    A = _entries(n, rowptr, col, val)
    senders_into = {j: [] for j in range(n)}    # N(j): k with A_jk != 0  (edge k -> j)
    for (i, j) in A:
        if i != j:
            senders_into[i].append(j)
    for j in senders_into:
        senders_into[j].sort()
    receivers_of = {j: [] for j in range(n)}   # i with A_ij != 0 (edge j -> i)
    for (i, j) in A:
        if i != j:
            receivers_of[j].append(i)
    for j in receivers_of:
        receivers_of[j].sort()
    if Lt is None:
        Lt = {(k, j): 0.0 for j in range(n) for k in senders_into[j]}
    if m is None:
        m = {(k, j): 0.0 for j in range(n) for k in senders_into[j]}
    x = [0.0] * n
    Sig = [0.0] * n
    for _ in range(sweeps):
        Lt_new, m_new = {}, {}
        for j in range(n):
            mj = b[j]
            Sj = A[(j, j)]
            for k in senders_into[j]:
                mj += m[(k, j)]
                Sj += Lt[(k, j)] * A.get((k, j), 0.0)
            x[j] = mj / Sj
            Sig[j] = Sj
            for i in receivers_of[j]:
                A_ij = A[(i, j)]
                back_L = Lt.get((i, j), 0.0)      # message i -> j exists iff A_ji != 0
                back_m = m.get((i, j), 0.0)
                L = -A_ij / (Sj - back_L * A_ij)
                Lt_new[(j, i)] = L
                m_new[(j, i)] = 0.0 if lambda_only else L * (mj - back_m)
        Lt, m = Lt_new, m_new
    return x, Lt, m, Sig


def conventional_gabp_loops(n, rowptr, col, val, b, sweeps):
    """Conventional GaBP in the (Lambda, mu) form of Sec. 2.2 (eq. GaBP_rules), flood schedule.

    Valid for matrices with a symmetric nonzero pattern (A_ji appears in a denominator).
    Returns the mean read-off mu_i of the last iteration.
    """
    A = _entries(n, rowptr, col, val)
    nbrs = {j: sorted(i for (jj, i) in A if jj == j and i != j) for j in range(n)}
    Lam = {(k, j): 0.0 for j in range(n) for k in nbrs[j]}
    mu = {(k, j): 0.0 for j in range(n) for k in nbrs[j]}
    x = [0.0] * n
    for _ in range(sweeps):
        for i in range(n):
            num = b[i] + sum(Lam[(j, i)] * mu[(j, i)] for j in nbrs[i])
            den = A[(i, i)] + sum(Lam[(j, i)] for j in nbrs[i])
            x[i] = num / den
        L2, m2 = {}, {}
        for j in range(n):
            for i in nbrs[j]:
                num = b[j] + sum(Lam[(k, j)] * mu[(k, j)] for k in nbrs[j] if k != i)
                den = A[(j, j)] + sum(Lam[(k, j)] for k in nbrs[j] if k != i)
                m2[(j, i)] = num / A[(j, i)]
                L2[(j, i)] = -A[(i, j)] * A[(j, i)] / den
        Lam, mu = L2, m2
    return x
