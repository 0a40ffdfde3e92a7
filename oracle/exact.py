"""Exact rational UniFrac for tiny inputs (pure Python, fractions.Fraction).

TEST INFRASTRUCTURE ONLY, used to pin the FP64 oracle.  It is written from the published
UniFrac definitions in a formulation that differs on purpose from uf_oracle.c:

* which tips lie under a branch is found from explicit descendant-tip sets (a depth-first
  walk down the children lists), not by walking reads up to the root;
* unweighted UniFrac is the branch length observed in exactly one of the two samples
  divided by the branch length observed in either (Lozupone & Knight 2005);
* weighted normalized UniFrac is sum_b L_b |A_b/A_T - B_b/B_T| divided by the normalizer
  sum_tips d_tip (A_tip/A_T + B_tip/B_T), with d_tip the root-to-tip distance
  (Lozupone et al. 2007).  The branch-by-branch denominator used by uf_oracle.c equals this
  normalizer in exact arithmetic, so agreement pins both.

Lengths may be floats (converted exactly with Fraction(float)) or Fractions.
"""
from __future__ import annotations

from fractions import Fraction


def _children(parent):
    ch = [[] for _ in parent]
    root = None
    for v, p in enumerate(parent):
        if p < 0:
            root = v
        else:
            ch[p].append(v)
    return ch, root


def _tips_below(parent):
    ch, root = _children(parent)
    below = [None] * len(parent)

    def walk(v):
        if not ch[v]:
            below[v] = frozenset([v])
        else:
            s = set()
            for c in ch[v]:
                walk(c)
                s |= below[c]
            below[v] = frozenset(s)

    walk(root)
    return ch, root, below


def _root_distance(parent, lengths, v):
    d = Fraction(0)
    while parent[v] >= 0:
        d += lengths[v]
        v = parent[v]
    return d


def _node_table(table_rows, feature_node, n_nodes):
    """table_rows: list of {feature: count}.  Returns per-sample {node: count}."""
    out = []
    for row in table_rows:
        m = {}
        for f, c in row.items():
            v = feature_node[f] if feature_node is not None else f
            m[v] = m.get(v, 0) + c
        out.append(m)
    return out


def unweighted(parent, length, table_rows, feature_node=None):
    """Condensed exact unweighted UniFrac (list of Fractions, squareform order)."""
    L = [Fraction(x) for x in length]
    ch, root, below = _tips_below(parent)
    rows = _node_table(table_rows, feature_node, len(parent))
    present = [{t for t, c in r.items() if c > 0} for r in rows]
    n = len(rows)
    out = []
    for i in range(n):
        for j in range(i + 1, n):
            unique = Fraction(0)
            observed = Fraction(0)
            for v in range(len(parent)):
                if v == root:
                    continue
                a = bool(below[v] & present[i])
                b = bool(below[v] & present[j])
                if a or b:
                    observed += L[v]
                if a != b:
                    unique += L[v]
            out.append(Fraction(0) if observed == 0 else unique / observed)
    return out


def weighted_normalized(parent, length, table_rows, feature_node=None):
    """Condensed exact weighted normalized UniFrac (list of Fractions, squareform order)."""
    L = [Fraction(x) for x in length]
    ch, root, below = _tips_below(parent)
    rows = _node_table(table_rows, feature_node, len(parent))
    totals = [sum(r.values()) for r in rows]
    tips = [v for v in range(len(parent)) if not ch[v]]
    dtip = {t: _root_distance(parent, L, t) for t in tips}
    n = len(rows)
    out = []
    for i in range(n):
        for j in range(i + 1, n):
            A, B = rows[i], rows[j]
            AT, BT = Fraction(totals[i]), Fraction(totals[j])
            u = Fraction(0)
            for v in range(len(parent)):
                if v == root:
                    continue
                Ab = sum(A.get(t, 0) for t in below[v])
                Bb = sum(B.get(t, 0) for t in below[v])
                u += L[v] * abs(Fraction(Ab) / AT - Fraction(Bb) / BT)
            norm = sum(dtip[t] * (Fraction(A.get(t, 0)) / AT + Fraction(B.get(t, 0)) / BT)
                       for t in tips)
            out.append(Fraction(0) if norm == 0 else u / norm)
    return out


def subtree_counts(parent, table_rows, feature_node=None):
    """Exact [n_samples][n_nodes] counts from descendant-tip sets."""
    ch, root, below = _tips_below(parent)
    rows = _node_table(table_rows, feature_node, len(parent))
    return [[sum(r.get(t, 0) for t in below[v]) for v in range(len(parent))] for r in rows]


def weighted_unnormalized(parent, length, table_rows, feature_node=None):
    """Condensed exact weighted unnormalized UniFrac: sum_b L_b |A_b/A_T - B_b/B_T|."""
    L = [Fraction(x) for x in length]
    ch, root, below = _tips_below(parent)
    rows = _node_table(table_rows, feature_node, len(parent))
    totals = [sum(r.values()) for r in rows]
    n = len(rows)
    out = []
    for i in range(n):
        for j in range(i + 1, n):
            A, B = rows[i], rows[j]
            AT, BT = Fraction(totals[i]), Fraction(totals[j])
            u = Fraction(0)
            for v in range(len(parent)):
                if v == root:
                    continue
                Ab = sum(A.get(t, 0) for t in below[v])
                Bb = sum(B.get(t, 0) for t in below[v])
                u += L[v] * abs(Fraction(Ab) / AT - Fraction(Bb) / BT)
            out.append(u)
    return out
