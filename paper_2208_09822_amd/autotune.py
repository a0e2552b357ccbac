"""Install-time autotuner of the tile table (the GPU form of the paper's
install-time / run-time split, Section III).

The run-time tiler's plan for (layout, m, n) is looked up in a table built at
install time.  The built-in plans follow fixed rules; this tuner measures,
on the device, alternatives for each class of shapes with the batched
kernel (the form the table serves), and records the fastest:

* matrix-core region (m, n > 8): how the ceil(m/16) x ceil(n/16) tiles are
  grouped into blocks (gm x gn groups, each at most 3 x 3 tiles), per
  (layout, tile rows, tile columns).  Grouping changes which wavefront
  computes a tile, never a tile's arithmetic, so results are bitwise the
  same for every choice;
* skinny region (m <= 8 or n <= 8): the built-in row strip, column strip or
  K-split block against matrix-core tiles, per (layout, m or n, tiles of
  the other side).

The result is a small text file (one line per class); ``apply`` turns it
into plans with iaat_plan_set / iaat_table_commit.  Timing uses seeded
synthetic problems drawn with a seed of their own (never the evaluation
data).

    python -m paper_2208_09822_amd.autotune --out paper_2208_09822_amd/tables/gfx950.txt
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

from . import iaat, inputs

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tables", "gfx950.txt")
TUNE_SEED = inputs.SEED_BASE + 77
LAYOUTS = ("NN", "TN", "NT", "TT")  # index = layout bits


def _kids():
    out = {}
    for kid in range(iaat.iaat_family_size()):
        info = iaat.iaat_family_info(kid)
        out[(info["family"], info["p1"], info["p2"])] = kid
    return out


def _groups(t, g):
    """t tiles in g balanced groups (largest first)."""
    return [t // g + (1 if i < t % g else 0) for i in range(g)]


def mfma_blocks(m, n, gm, gn, kids):
    tm, tn = -(-m // 16), -(-n // 16)
    blocks, r0 = [], 0
    for a in _groups(tm, gm):
        c0 = 0
        for b in _groups(tn, gn):
            blocks.append((16 * r0, 16 * c0, kids[("MFMA", a, b)]))
            c0 += b
        r0 += a
    return blocks


def class_of(layout, m, n):
    """Shape class and the choices tried for it."""
    tm, tn = -(-m // 16), -(-n // 16)
    mf = ["mfma:%d:%d" % (gm, gn) for gm in range(-(-tm // 3), tm + 1)
          for gn in range(-(-tn // 3), tn + 1) if gm * gn <= 15]
    if m <= 4 and n <= 4:
        return ("kred", layout, m, n), ["default"] + mf
    if m <= 8:
        return ("rows", layout, m, tn), ["default"] + mf
    if n <= 8:
        return ("cols", layout, n, tm), ["default"] + mf
    return ("mfma", layout, tm, tn), mf


def representative(key):
    kind, layout, a, b = key
    if kind == "kred":
        return a, b
    if kind == "rows":
        return a, min(16 * b, 80)
    if kind == "cols":
        return min(16 * b, 80), a
    return min(16 * a, 80), min(16 * b, 80)


def plan_for(choice, m, n, kids):
    if choice == "default":
        return None
    _, gm, gn = choice.split(":")
    return mfma_blocks(m, n, int(gm), int(gn), kids)


def _time_batch(ctx, torch, dev, layout, m, n, reps):
    lay = LAYOUTS[layout]
    kmax = 32768 if lay == "TN" else 512000
    k = max(1, min(48, kmax // (m * n)))
    per = 4 * (m * k + k * n + 2 * m * n)
    count = int(min(16384, max(1024, (16 << 20) // per)))
    ps = inputs.uniform_problems([(lay, m, n, k)] * count, seed=TUNE_SEED + 7 * m + n,
                                 alpha=1.0, beta=1.0)
    buf = torch.from_numpy(ps.buf).to(dev)
    d = torch.from_numpy(iaat.descriptors(ps, buf.data_ptr()).view(np.uint8)).to(dev)
    s = torch.cuda.current_stream(dev)
    # the graph-replayed batched launch, the form the tuned table serves
    plan = iaat.iaat_vbplan_create(ctx, d.data_ptr(), count)

    def run():
        iaat.iaat_vbplan_launch(plan, s.cuda_stream)

    def measure():
        run()
        torch.cuda.synchronize(dev)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(reps):
            run()
        b.record(s)
        torch.cuda.synchronize(dev)
        return a.elapsed_time(b) / reps
    measure.plan = plan
    return measure


def tune(out_path, reps=5, verbose=True):
    import torch
    dev = torch.device("cuda:0")
    ctx = iaat.Context(0)
    kids = _kids()
    classes = {}
    for layout in range(4):
        for m in range(1, 81):
            for n in range(1, 81):
                key, choices = class_of(layout, m, n)
                classes.setdefault(key, choices)
    lines = ["# Tile-table tuning for gfx950: fastest plan choice per shape class,",
             "# measured with the batched kernel by paper_2208_09822_amd/autotune.py.",
             "# kind layout a b choice us(choice) us(first choice)"]
    t0 = time.time()
    for key in sorted(classes):
        m, n = representative(key)
        layout = key[1]
        measure = _time_batch(ctx.handle, torch, dev, layout, m, n, reps)
        best, best_t, first_t = None, math.inf, None
        for choice in classes[key]:
            blocks = plan_for(choice, m, n, kids)
            if blocks is None:
                blocks = [(b[0], b[1], b[4]) for b in iaat.iaat_default_plan(layout, m, n)]
            iaat.iaat_plan_set(ctx.handle, layout, m, n, blocks)
            iaat.iaat_table_commit(ctx.handle)
            t = measure()
            if first_t is None:
                first_t = t
            if t < best_t:
                best, best_t = choice, t
        iaat.iaat_vbplan_destroy(measure.plan)
        lines.append("%s %d %d %d %s %.2f %.2f" % (key[0], key[1], key[2], key[3], best,
                                                   best_t * 1e3, first_t * 1e3))
        if verbose:
            print("[tune] %-24s best %-10s %8.2f us (first %8.2f us)  %.0fs" % (
                str(key), best, best_t * 1e3, first_t * 1e3, time.time() - t0), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(out_path)), exist_ok=True)
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    ctx.close()
    return out_path


def load(path):
    choices = {}
    for line in open(path):
        line = line.split("#")[0].split()
        if line:
            choices[(line[0], int(line[1]), int(line[2]), int(line[3]))] = line[4]
    return choices


def apply(ctx, path=DEFAULT_TABLE):
    """Stage and commit the tuned plans of `path` into context `ctx`;
    returns the number of plans changed."""
    choices = load(path)
    kids = _kids()
    changed = 0
    for layout in range(4):
        for m in range(1, 81):
            for n in range(1, 81):
                key, _ = class_of(layout, m, n)
                blocks = plan_for(choices.get(key, "default"), m, n, kids)
                if blocks is not None:
                    iaat.iaat_plan_set(ctx, layout, m, n, blocks)
                    changed += 1
    iaat.iaat_table_commit(ctx)
    return changed


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    tune(args.out, reps=args.reps)
    return 0


if __name__ == "__main__":
    sys.exit(main())
