"""Query rewriting (Section 6.1), derived and executed literally -- TEST INFRASTRUCTURE ONLY.

Generic Join's loop for X_sigma(i) intersects one operand per atom that holds
the variable; the operand of atom j is its X_sigma(i) column restricted by the
values of the atom's other variables bound in enclosing loops.  Call d_j the
deepest level among those variables (0 when none is bound: then the operand
is the atom's whole column).  An operand with d_j < i-1 does not change while
the loop at level i-1 iterates, so it is recomputed needlessly for every
iteration.  The rewriting lifts those operands: when at least two operands of
level i have d_j < i-1, their intersection is computed once, right after the
variable of level L = max d_j is bound (L = 0: before the outermost loop), and
stored as a sorted temporary array tmp; the loop at level i then intersects
tmp with the remaining operands.  This is the reading of "the general case
follows immediately" taken here; the paper's 4-clique example (Figure
"Example of Query Rewriting") is its instance: tmp_Y at level 0, tmp_Z after
x, tmp_U after y.  Only one lift per level and no nested lifts.

Soundness rests on intersection being associative and commutative on sorted
sets (Figure "Simplified Pseudocode"): the rewritten program returns exactly
the original result.  ``run_rewritten`` executes the lifted program with
Python sets and sorted lists, for small inputs only.
"""

from __future__ import annotations

from collections import defaultdict


def derive_plan(n_vars: int, atoms, order):
    """Per level (1-based): list of (atom, dep) operands and the lifted group.

    Returns dict with
      levels[i] = {"var": X, "ops": [(atom, dep), ...], "lift": None or (L, [atoms])}
    """
    pos = {v: i + 1 for i, v in enumerate(order)}
    levels = {}
    for i, x in enumerate(order, start=1):
        ops = []
        for j, a in enumerate(atoms):
            if x not in a:
                continue
            dep = max([pos[v] for v in a if pos[v] < i], default=0)
            ops.append((j, dep))
        low = [(j, d) for j, d in ops if d < i - 1]
        lift = None
        if len(low) >= 2:
            lift = (max(d for _, d in low), sorted(j for j, _ in low))
        levels[i] = {"var": x, "ops": ops, "lift": lift}
    return levels


def _operand_index(n_vars, atoms, relations, order):
    """idx[(j, x)][prefix tuple] -> sorted list of x values, prefix = atom j's variables
    bound before x (in variable order)."""
    pos = {v: i for i, v in enumerate(order)}
    idx = {}
    for j, (a, rel) in enumerate(zip(atoms, relations)):
        rows = set(map(tuple, rel))
        for c, x in enumerate(a):
            before = sorted([cc for cc, v in enumerate(a) if pos[v] < pos[x]], key=lambda cc: pos[a[cc]])
            d = defaultdict(set)
            for row in rows:
                d[tuple(row[cc] for cc in before)].add(row[c])
            idx[(j, x)] = ({k: sorted(v) for k, v in d.items()}, before)
    return idx


def _intersect(lists):
    if not lists:
        return []
    s = set(lists[0])
    for l in lists[1:]:
        s &= set(l)
    return sorted(s)


def run_rewritten(n_vars: int, atoms, relations, order, rewrite=True):
    """Count and sorted head-order rows of the (optionally rewritten) GJ program."""
    relations = [[tuple(int(x) for x in r) for r in rel] for rel in relations]
    plan = derive_plan(n_vars, atoms, order)
    idx = _operand_index(n_vars, atoms, relations, order)
    n = len(order)
    out = []
    val = {}

    def operand(j, x):
        table, before = idx[(j, x)]
        key = tuple(val[atoms[j][cc]] for cc in before)
        return table.get(key, [])

    def lifts_at(L):
        return [i for i in range(1, n + 1) if rewrite and plan[i]["lift"] and plan[i]["lift"][0] == L]

    def level(i, tmps):
        if i > n:
            out.append(tuple(val[v] for v in range(n_vars)))
            return
        x = plan[i]["var"]
        lists = []
        lifted = set(plan[i]["lift"][1]) if (rewrite and plan[i]["lift"]) else set()
        for j, _ in plan[i]["ops"]:
            if j not in lifted:
                lists.append(operand(j, x))
        if lifted:
            lists.append(tmps[i])
        for v in _intersect(lists):
            val[x] = v
            t2 = dict(tmps)
            for k in lifts_at(i):
                t2[k] = _intersect([operand(j, plan[k]["var"]) for j in plan[k]["lift"][1]])
            level(i + 1, t2)
        val.pop(x, None)

    tmps0 = {}
    for k in lifts_at(0):
        tmps0[k] = _intersect([operand(j, plan[k]["var"]) for j in plan[k]["lift"][1]])
    level(1, tmps0)
    out.sort()
    return len(out), out
