"""Plain-loop brute force of coarse-to-fine surface localization (Sec. 3.2), used to pin
the oracle.  It is written independently of the oracle: dictionaries over node
tuples, explicit corner enumeration and a randomized work list for the conflict
closure (whose least fixed point does not depend on the order)."""
import itertools
import math
import random


def _sig(lg):
    if lg == -math.inf:
        return 0.0
    return 1.0 / (1.0 + math.exp(-lg)) if lg > -700 else 0.0


def brute_localize(logit_fn, n0, T, seed):
    """Independent implementation with plain loops and a randomized work list.

    n0 is the coarsest level's cell count per axis: an int (cube) or a tuple
    (cx, cy, cz) for an anisotropic lattice such as the render's; every level
    doubles all three.  Returns per-level sets of evaluated (i, j, k) on each
    level's lattice, the final labels, the final cell counts, the final values
    (sigmoid of the logit where evaluated, else the interpolated 0/1) and the set
    of nodes evaluated at any level.
    """
    rnd = random.Random(seed)
    cells = tuple(n0) if isinstance(n0, (tuple, list)) else (n0, n0, n0)
    nodes = list(itertools.product(*(range(c + 1) for c in cells)))
    coord = lambda q, c: tuple(-1.0 + 2.0 * x / n for x, n in zip(q, c))
    lg0 = {q: logit_fn(coord(q, cells)) for q in nodes}
    label = {q: int(lg0[q] > 0) for q in nodes}
    val = {q: _sig(lg0[q]) for q in nodes}
    done = set(nodes)
    per_level = [set(nodes)]
    for t in range(1, T + 1):
        cells = tuple(2 * c for c in cells)
        new_label = {}
        new_val = {}
        interp = {}
        new_done = set()
        for q in itertools.product(*(range(c + 1) for c in cells)):
            corners = list(itertools.product(*[sorted({x // 2, (x + 1) // 2}) for x in q]))
            vals = [label[c] for c in corners]
            interp[q] = sum(vals) / len(vals)
            if all(x % 2 == 0 for x in q):
                new_label[q] = label[tuple(x // 2 for x in q)]
                new_val[q] = val[tuple(x // 2 for x in q)]
                if tuple(x // 2 for x in q) in done:
                    new_done.add(q)
            else:
                new_label[q] = 1 if interp[q] > 0.5 else 0
                new_val[q] = interp[q]
        nb = lambda q: [(q[0] + a, q[1] + b, q[2] + c) for a in (-1, 0, 1) for b in (-1, 0, 1)
                        for c in (-1, 0, 1)
                        if 0 <= q[0] + a <= cells[0] and 0 <= q[1] + b <= cells[1]
                        and 0 <= q[2] + c <= cells[2]]
        b0 = [q for q in interp if 0 < interp[q] < 1]
        work = sorted({w for q in b0 for w in nb(q) if w not in new_done})
        rnd.shuffle(work)
        queued = set(work)
        evaluated_here = set()
        while work:
            q = work.pop()
            lg = logit_fn(coord(q, cells))
            new_label[q] = int(lg > 0)
            new_val[q] = _sig(lg)
            new_done.add(q)
            evaluated_here.add(q)
            if new_label[q] != int(interp[q] > 0.5):
                for w in nb(q):
                    if w not in new_done and w not in queued:
                        queued.add(w)
                        work.insert(rnd.randrange(len(work) + 1), w)
        label = new_label
        val = new_val
        done = new_done
        per_level.append(evaluated_here)
    return per_level, label, cells, val, done
