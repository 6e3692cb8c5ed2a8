"""Loader for the paper's running example (Sec. 2.1, Tables 2-4), stored in
tests/golden/worked_example.json with its citation."""
import json
import os

import numpy as np

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "worked_example.json")


def load():
    with open(_PATH) as f:
        g = json.load(f)
    alpha = {c: i for i, c in enumerate(g["alphabet"])}
    q = g["q"]
    b = 2
    # Table 2 values in (0,1) become u64 fixed-point ranks (order is all that matters);
    # q-grams absent from Table 2 never occur in the five strings.
    table = np.full(1 << (b * q), np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    for gram, v in g["pi_table"].items():
        code = 0
        for c in gram:
            code = (code << b) | alpha[c]
        table[code] = np.uint64(int(round(v * 100)))
    strings = [np.array([alpha[c] for c in s], dtype=np.uint8) for s in g["strings"]]
    offsets = np.zeros(len(strings) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(s) for s in strings])
    chars = np.concatenate(strings)
    return g, table, strings, chars, offsets


def pairs_1based(arr):
    return [[int(v >> np.uint64(32)) + 1, int(v & np.uint64(0xFFFFFFFF)) + 1] for v in arr]
