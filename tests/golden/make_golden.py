"""Writes the stored expected values under tests/golden/ that are not taken
from a publication.  It calls only the oracle (``oracle/``) and the input
generators (``synth``), never the HIP library.

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth   # noqa: E402


def permute_fixture():
    base = synth.base_labels([5, 4, 7])
    perms = oracle.permute(base, 4, seed=3000)
    path = os.path.join(HERE, "permute_n16_P4_seed3000.txt")
    with open(path, "w") as f:
        f.write("# Fisher-Yates shuffles of the base labels (first row) with the\n"
                "# per-permutation SplitMix64 streams of seed 3000; written by\n"
                "# make_golden.py from the oracle.  Rows 2.. are permutations 0..3.\n")
        f.write(" ".join(map(str, base.tolist())) + "\n")
        for row in perms:
            f.write(" ".join(map(str, row.tolist())) + "\n")


if __name__ == "__main__":
    permute_fixture()
