"""Writes the stored known-answer fixtures of this folder.

Calls only the FP64 oracle (``oracle/``).  Run from the repository root:
``python -m tests.golden.make_golden``.

crn_known_answers.txt: the shared Monte Carlo draws (u, z0, z1, z2) of a
few (seed, pass, S) blocks, as float32 bit patterns in hex, so that any
implementation of the draw generator can be compared bit for bit.
"""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CRN_FILE = os.path.join(HERE, "crn_known_answers.txt")
CRN_CASES = [(0, 0, 1), (0, 1, 1), (0, 7, 4), (1, 0, 8), (12345, 3, 2),
             (0xFFFFFFFFFFFFFFFF, 1000, 3)]


def write_crn_golden():
    from oracle import crn_block
    lines = ["# seed round S : float32 hex words of the [S,4] block (u z0 z1 z2 ...)"]
    for seed, r, S in CRN_CASES:
        blk = crn_block(seed, r, S)
        words = " ".join(f"{w:08x}" for w in blk.view(np.uint32).reshape(-1))
        lines.append(f"{seed} {r} {S} : {words}")
    with open(CRN_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def load_crn_golden():
    out = {}
    with open(CRN_FILE) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            head, words = line.split(":")
            seed, r, S = (int(x) for x in head.split())
            vals = np.array([int(w, 16) for w in words.split()], dtype=np.uint32)
            out[(seed, r, S)] = vals.view(np.float32).reshape(S, 4)
    return out


if __name__ == "__main__":
    write_crn_golden()
