"""Writes gpu_strip_dp.txt: for every M, N in 1..80, the strip-DP optimum of
the memory-operation cost S = sum of (m_i + n_i) over the blocks of a tiling
(the K coefficient of Section V-A's load count), over the GPU kernel
family's block heights.  A strip of height h may be cut from any family
block at least h rows tall (edge blocks are clipped), so its widest piece is
64 columns for h <= 8 (row strips), 48 for h <= 48 (3 x 3 grids of 16 x 16
matrix-core tiles), 8 for h <= 64 (column strips).  Calls only the oracle.

    python tests/golden/make_gpu_strip_dp.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tiler_ref  # noqa: E402

GPU_NMAX = {h: (64 if h <= 8 else 48 if h <= 48 else 8) for h in range(1, 65)}


def main():
    lines = ["# Strip-DP optimum of S = sum(m_i + n_i) over the GPU family's strip heights",
             "# (Section V-A cost model; see make_gpu_strip_dp.py).  Columns: M N S_opt"]
    for m in range(1, 81):
        for n in range(1, 81):
            lines.append("%d %d %d" % (m, n, tiler_ref.strip_dp_optimum(m, n, GPU_NMAX)))
    with open(os.path.join(HERE, "gpu_strip_dp.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
