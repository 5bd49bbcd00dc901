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

Per output that is 4 x 32 (row sorts) + 2 x 42 + 100 + 2 x 72 + 4 x 14 = 512
min/max operations per four outputs, 128 per output.

All merges are Batcher odd-even merges (lists padded to a power of two with
+inf) pruned symbolically to the outputs needed; comparisons against a
constant +inf vanish and only the min or max side of a comparator that is
used is emitted.  CG_SORT7 is the 16-comparator 7-input sorting network.  The
script checks the composed networks against numpy's median on random inputs
with ties before writing the file.
"""

import os
import sys

import numpy as np

SORT7 = [(0, 6), (2, 3), (4, 5), (0, 2), (1, 4), (3, 6), (0, 1), (2, 5), (3, 4),
         (1, 2), (4, 6), (2, 3), (4, 5), (1, 2), (3, 4), (5, 6)]
INF = -1


def _check_sort7():
    for bits in range(128):
        v = [(bits >> i) & 1 for i in range(7)]
        for a, b in SORT7:
            if v[a] > v[b]:
                v[a], v[b] = v[b], v[a]
        assert v == sorted(v), bits


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


def evaluate(kept, outs, vals):
    env = {i: vals[:, i] for i in range(vals.shape[1])}
    for nid, op, a, b in kept:
        env[nid] = np.minimum(env[a], env[b]) if op == "min" else np.maximum(env[a], env[b])
    return np.stack([env[o] for o in outs], axis=1)


def emit(name, kept, outs, n_in, in_name="IN", out_name="OUT"):
    lines = [f"// {name}: {len(kept)} min/max operations",
             f"#define {name}({in_name}, {out_name}) do {{ \\"]
    for nid, op, a, b in kept:
        sa = f"{in_name}[{a}]" if a < n_in else f"_t{a}"
        sb = f"{in_name}[{b}]" if b < n_in else f"_t{b}"
        fn = "fminf" if op == "min" else "fmaxf"
        lines.append(f"  const float _t{nid} = {fn}({sa}, {sb}); \\")
    for j, o in enumerate(outs):
        src = f"{in_name}[{o}]" if o < n_in else f"_t{o}"
        lines.append(f"  {out_name}[{j}] = {src}; \\")
    lines.append("} while (0)")
    return "\n".join(lines) + "\n"


def emit_sort7(name):
    lines = [f"// {name}: 16 compare-exchanges, sorts V[0..6] ascending",
             f"#define {name}(V) do {{ \\"]
    for a, b in SORT7:
        lines.append(f"  {{ const float _lo = fminf(V[{a}], V[{b}]); "
                     f"V[{b}] = fmaxf(V[{a}], V[{b}]); V[{a}] = _lo; }} \\")
    lines.append("} while (0)")
    return "\n".join(lines) + "\n"


def main(path):
    _check_sort7()
    k77, o77 = merge_select([7, 7], list(range(14)))
    kc, oc = merge_select([14, 14], list(range(3, 25)))
    kp, op = merge_select([22, 14], list(range(14, 22)))
    kf, of = merge_select([8, 7], [7])
    rng = np.random.default_rng(0)
    for trial in range(4):
        v = rng.random((20000, 70)) if trial % 2 == 0 else \
            rng.integers(0, 5, size=(20000, 70)).astype(np.float64)
        rows = np.sort(v.reshape(-1, 10, 7), axis=2)  # rows t .. t+9, each sorted
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
