"""Generate the branch-free 7x7 median selection networks used by the HIP kernels.

Build step (run by paper_2307_12988_amd/build.py; output median49_net.inc).

The median of a 7x7 window is the 25th smallest of its 49 values.  The kernel
sorts each 7-value row segment of the image once and walks down the frames
computing four vertically adjacent windows at a time, W0..W3 over rows
t..t+6, t+1..t+7, t+2..t+8 and t+3..t+9.  With L1..L4 the merged row pairs
(t+1, t+2), (t+3, t+4), (t+5, t+6), (t+7, t+8):

* W0 and W1 share the 42 values of L1, L2, L3; W2 and W3 those of L2, L3, L4.
  At most 7 values of a window's own row can fall below or above, so only
  ranks 17..24 of a shared set can be the median: the median is the 8th
  smallest of those 8 values together with the own row (CG_MERGE8_7_R7).
* L2 and L3 (28 values) are common to both shared sets.  A shared set adds 14
  values (L1 or L4) to them, so its ranks 17..24 only need ranks 3..24 of
  the common part (CG_CORE_R3_24): the 3 smallest dropped values lie at rank
  <= 16 of the shared set and the 3 largest at rank >= 25.  Ranks 17..24 of
  the shared set are then ranks 14..21 of those 22 values merged with L1 or
  L4 (CG_PAIR_R14_21).
* L3 and L4 of one step are L1 and L2 of the next (t + 4), so each step merges
  two new row pairs (CG_MERGE77) and sorts four new rows.

All merges are Batcher odd-even merges (lists padded to a power of two with
+inf) pruned symbolically to the outputs needed; comparisons against a
constant +inf vanish and only the min or max side of a comparator that is
used is emitted.

The hardware has three-input min, max and median instructions at the rate of
the two-input ones, so two further rewrites pay:
* CG_SORT7 sorts three values with one min3, med3 and max3 and then inserts
  the other four one at a time; inserting x into a sorted list s gives
  min(x, s0), med3(s(j-1), x, s(j)) for the inner positions and
  max(x, s_last): 25 operations instead of the 32 of the best two-input
  network (16 comparators).  CG_MED7 keeps only the operations that the
  4th smallest needs (13 instructions): the bounds of the centre-only
  start, where a window's median lies between the smallest and the largest
  median of its seven row segments.
* In a pruned merge, max(min(a, b), c) equals med3(a, b, c) whenever c <= a
  or c <= b holds for every input, and min(max(a, b), c) does whenever
  a <= c or b <= c does; where the inner operation has no other use the two
  become one.  The conditions are proved by the 0-1 principle (every node is
  a monotone function of the inputs, so an order that holds on all 0-1
  inputs with sorted lists holds on all inputs).
The compiler fuses min(min(a, b), c) and max(max(...)) by itself.  Before
the rewrites a step took 4 x 32 (row sorts) + 2 x 42 + 100 + 2 x 72 + 4 x 14
= 512 min/max operations per four outputs (128 per output).

The script checks every network exhaustively on 0-1 inputs and the composed
networks against numpy's median on random inputs with ties before writing
the file.
"""

import os
import sys

import numpy as np

INF = -1


def _oe_merge(w):
    n = len(w)
    if n == 2:
        return [(w[0], w[1])]
    ops = _oe_merge(w[0::2]) + _oe_merge(w[1::2])
    for i in range(1, n - 1, 2):
        ops.append((w[i], w[i + 1]))
    return ops


def merge_select(list_lens, want_ranks):
    """Merge sorted lists (inputs numbered consecutively, list by list) with a
    Batcher merge tree and keep the operations the wanted ranks need.
    Returns (ops, outputs): ops are (id, 'min'|'max', a, b) in SSA order."""
    n_in = sum(list_lens)
    nodes = []
    counter = [n_in]
    n_lists = 1
    while n_lists < len(list_lens):
        n_lists *= 2
    per = 8
    while per < max(list_lens):
        per *= 2
    wires = [INF] * (n_lists * per)
    base = 0
    for li, ln in enumerate(list_lens):
        for r in range(ln):
            wires[li * per + r] = base + r
        base += ln

    def ce(i, j):
        a, b = wires[i], wires[j]
        if b == INF:
            return
        if a == INF:
            wires[i], wires[j] = b, INF
            return
        lo, hi = counter[0], counter[0] + 1
        counter[0] += 2
        nodes.append((lo, "min", a, b))
        nodes.append((hi, "max", a, b))
        wires[i], wires[j] = lo, hi

    size = per
    while size < n_lists * per:
        for start in range(0, n_lists * per, 2 * size):
            for i, j in _oe_merge(list(range(start, start + 2 * size))):
                ce(i, j)
        size *= 2
    outs = [wires[r] for r in want_ranks]
    live = set(outs)
    kept = []
    for nid, op, a, b in reversed(nodes):
        if nid in live:
            kept.append((nid, op, a, b))
            live.add(a)
            live.add(b)
    kept.reverse()
    return kept, outs


def _apply(op, x):
    if op == "min":
        return np.minimum(x[0], x[1])
    if op == "max":
        return np.maximum(x[0], x[1])
    lo, hi = np.minimum(x[0], x[1]), np.maximum(x[0], x[1])  # med3
    return np.maximum(lo, np.minimum(hi, x[2]))


def evaluate(kept, outs, vals):
    env = {i: vals[:, i] for i in range(vals.shape[1])}
    for nid, op, *args in kept:
        env[nid] = _apply(op, [env[a] for a in args])
    return np.stack([env[o] for o in outs], axis=1)


def zero_one_inputs(list_lens):
    """Every 0-1 input whose lists are each sorted ascending."""
    rows = []
    for zeros in np.ndindex(*[n + 1 for n in list_lens]):
        v = []
        for n, z in zip(list_lens, zeros):
            v += [0] * z + [1] * (n - z)
        rows.append(v)
    return np.array(rows, dtype=np.int8)


def fuse_med3(kept, outs, list_lens):
    """Replace max(min(a, b), c) by med3(a, b, c) where c <= a or c <= b on
    every sorted 0-1 input (and min(max(a, b), c) where a <= c or b <= c),
    when the inner operation has no other use."""
    n_in = sum(list_lens)
    zo = zero_one_inputs(list_lens)
    env = {i: zo[:, i] for i in range(n_in)}
    node = {}
    uses = {}
    for nid, op, a, b in kept:
        env[nid] = _apply(op, [env[a], env[b]])
        node[nid] = (op, a, b)
        uses[a] = uses.get(a, 0) + 1
        uses[b] = uses.get(b, 0) + 1
    for o in outs:
        uses[o] = uses.get(o, 0) + 1

    def le(x, y):
        return bool(np.all(env[x] <= env[y]))

    dead = set()
    new = {}
    for nid, op, a, b in kept:
        for p, c in ((a, b), (b, a)):
            if p not in node or p in dead or uses[p] != 1 or p in new:
                continue
            pop, pa, pb = node[p]
            if (op == "max" and pop == "min" and (le(c, pa) or le(c, pb))) or \
               (op == "min" and pop == "max" and (le(pa, c) or le(pb, c))):
                dead.add(p)
                new[nid] = (nid, "med3", pa, pb, c)
                break
    return [new.get(t[0], t) for t in kept if t[0] not in dead]


def check_zero_one(kept, outs, list_lens, want_ranks):
    """Exhaustive 0-1 check: the outputs are the wanted ranks of the merge."""
    zo = zero_one_inputs(list_lens)
    got = evaluate(kept, outs, zo)
    want = np.sort(zo, axis=1)[:, want_ranks]
    assert np.array_equal(got, want)


def sort7_ops():
    """Sort of V[0..6] (inputs 0..6) as SSA operations: min3/med3/max3 of the
    first three, then insertion of V[3] .. V[6]."""
    ops = []
    nid = [7]

    def put(op, *args):
        ops.append((nid[0], op) + args)
        nid[0] += 1
        return nid[0] - 1

    m = put("min", 0, 1)
    s = [put("min", m, 2), put("med3", 0, 1, 2), put("max", put("max", 0, 1), 2)]
    for x in range(3, 7):
        t = [put("min", x, s[0])]
        t += [put("med3", s[j - 1], x, s[j]) for j in range(1, len(s))]
        t.append(put("max", x, s[-1]))
        s = t
    return ops, s


def med7_ops():
    """The 4th smallest of V[0..6]: sort7_ops without the operations that
    output does not depend on."""
    ops, outs = sort7_ops()
    live = {outs[3]}
    kept = []
    for op in reversed(ops):
        if op[0] in live:
            kept.append(op)
            live.update(op[2:])
    return kept[::-1], [outs[3]]


def emit(name, kept, outs, n_in, in_name="IN", out_name="OUT"):
    lines = [f"// {name}: {len(kept)} min/max/med3 operations",
             f"#define {name}({in_name}, {out_name}) do {{ \\"]
    fns = {"min": "fminf", "max": "fmaxf", "med3": "__builtin_amdgcn_fmed3f"}
    for nid, op, *args in kept:
        srcs = ", ".join(f"{in_name}[{a}]" if a < n_in else f"_t{a}" for a in args)
        lines.append(f"  const float _t{nid} = {fns[op]}({srcs}); \\")
    for j, o in enumerate(outs):
        src = f"{in_name}[{o}]" if o < n_in else f"_t{o}"
        lines.append(f"  {out_name}[{j}] = {src}; \\")
    lines.append("} while (0)")
    return "\n".join(lines) + "\n"


def emit_sort7(name):
    ops, outs = sort7_ops()
    # in place: the outputs overwrite the inputs only after every temporary
    # is formed
    text = emit(name, ops, outs, 7, "V", "V")
    text = text.replace(f"#define {name}(V, V)", f"#define {name}(V)", 1)
    return text.replace(f"// {name}: ", f"// {name}: sorts V[0..6] ascending in place, ", 1)


def main(path):
    s7, s7o = sort7_ops()
    zo = np.array([[(bits >> i) & 1 for i in range(7)] for bits in range(128)], dtype=np.int8)
    assert np.array_equal(evaluate(s7, s7o, zo), np.sort(zo, axis=1))
    m7, m7o = med7_ops()
    assert np.array_equal(evaluate(m7, m7o, zo)[:, 0], np.sort(zo, axis=1)[:, 3])
    nets = {}
    for name, lens, ranks in (("k77", [7, 7], list(range(14))),
                              ("kc", [14, 14], list(range(3, 25))),
                              ("kp", [22, 14], list(range(14, 22))),
                              ("kf", [8, 7], [7])):
        kept, outs = merge_select(lens, ranks)
        kept = fuse_med3(kept, outs, lens)
        check_zero_one(kept, outs, lens, ranks)
        nets[name] = (kept, outs)
    (k77, o77), (kc, oc), (kp, op), (kf, of) = nets["k77"], nets["kc"], nets["kp"], nets["kf"]
    rng = np.random.default_rng(0)
    for trial in range(4):
        v = rng.random((20000, 70)) if trial % 2 == 0 else \
            rng.integers(0, 5, size=(20000, 70)).astype(np.float64)
        raw = v.reshape(-1, 10, 7)
        rows = np.stack([evaluate(s7, s7o, raw[:, j]) for j in range(10)], axis=1)
        assert np.array_equal(rows, np.sort(raw, axis=2))  # rows t .. t+9, each sorted
        lists = [evaluate(k77, o77, np.concatenate([rows[:, 2 * j + 1], rows[:, 2 * j + 2]],
                                                   axis=1)) for j in range(4)]
        core = evaluate(kc, oc, np.concatenate([lists[1], lists[2]], axis=1))
        sa = evaluate(kp, op, np.concatenate([core, lists[0]], axis=1))
        sb = evaluate(kp, op, np.concatenate([core, lists[3]], axis=1))
        for w, (shared, own) in enumerate([(sa, 0), (sa, 7), (sb, 2), (sb, 9)]):
            got = evaluate(kf, of, np.concatenate([shared, rows[:, own]], axis=1))[:, 0]
            want = np.sort(v.reshape(-1, 10, 7)[:, w:w + 7].reshape(-1, 49), axis=1)[:, 24]
            assert np.array_equal(got, want), (trial, w)
    text = ["// Generated by gen_median_net.py -- do not edit.", ""]
    text.append(emit_sort7("CG_SORT7"))
    text.append(emit("CG_MED7", m7, m7o, 7, "V", "OUT"))
    text.append(emit("CG_MERGE77", k77, o77, 14))
    text.append(emit("CG_CORE_R3_24", kc, oc, 28))
    text.append(emit("CG_PAIR_R14_21", kp, op, 36))
    text.append(emit("CG_MERGE8_7_R7", kf, of, 15))
    with open(path, "w") as fh:
        fh.write("\n".join(text))
    return 0


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    sys.exit(main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, "median49_net.inc")))
