"""Write expected bootstrap outputs for workloads too large for the oracle to
run inside a GPU test, by running the oracle (and nothing else) on the seeded
draws that the test regenerates.

    python tests/golden/make_oracle_expected.py [name ...]

Each set below names its parameters, seeds and sampled ciphertext indices; the
file it writes holds one line per sampled ciphertext: the index, then the n + 1
output words.  Only ``oracle`` and ``synth`` (seeded draws) are used.
"""
from __future__ import annotations

import os
import sys
import time
from dataclasses import replace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import PRESETS, enc_draws, key_draws, messages, negacyclic_table  # noqa: E402

# The TFHE-shaped comparison point for t = 2^14 (Sec. 1 comparison table, Sec. 5
# Tables 1-2): one ring of degree N r = 8192 with r = 1, the paper-shaped n,
# gadget and key switch; the batch of 4096 ciphertexts that the benchmark's
# comparison leg times, of which the listed indices are computed here.
SETS = {
    "tfhe_shaped_8192": dict(
        params=replace(PRESETS["paper_shaped"]["params"], N=8192),
        key_seed=1, t=16384, r=1, table_seed=103, enc_seed=703, msg_seed=704, batch=4096,
        pick=(0, 4095),
    ),
}


def path(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.txt")


def inputs(spec: dict, s: np.ndarray):
    """The set's batch as the oracle encrypts it from the draws."""
    p, t, r = spec["params"], spec["t"], spec["r"]
    q = 2 * p.N * r
    ed = enc_draws(p.n, q, spec["batch"], spec["enc_seed"])
    m = messages(t, spec["batch"], spec["msg_seed"])
    return q, m, oracle.encrypt(p.n, q, t, s, m, ed["a"], ed["e"])


def make(name: str) -> None:
    spec = SETS[name]
    p, t, r = spec["params"], spec["t"], spec["r"]
    t0 = time.time()
    keys = oracle.KeySet(p, key_draws(p, spec["key_seed"]))
    f = negacyclic_table(t, t, spec["table_seed"])
    V = oracle.test_vector(p.N, r, p.Q, t, t, f)
    q, m, ct = inputs(spec, keys.s)
    pick = np.array(spec["pick"])
    print(f"{name}: keys in {time.time() - t0:.0f} s; oracle on {pick.size} ciphertexts", flush=True)
    out = oracle.bootstrap_many(p, r, keys.bsk, keys.ksk, V, q, q, ct[pick])
    with open(path(name), "w") as fh:
        fh.write(f"# Written by tests/golden/make_oracle_expected.py ({name}) from the oracle alone.\n")
        fh.write(f"# n={p.n} N={p.N} Q={p.Q} log2_B={p.log2_B} l={p.l} log2_Bks={p.log2_Bks} l_ks={p.l_ks} "
                 f"ternary={int(p.ternary)} t={t} r={r} q_in=q_out={q}\n")
        fh.write(f"# seeds: keys {spec['key_seed']}, table {spec['table_seed']}, encryption {spec['enc_seed']}, "
                 f"messages {spec['msg_seed']}; batch {spec['batch']}\n")
        fh.write("# line: ciphertext index, then the n + 1 output words\n")
        for k, i in enumerate(pick):
            fh.write(f"{int(i)} " + " ".join(str(int(v)) for v in out[k]) + "\n")
    print(f"{name}: wrote {path(name)} in {time.time() - t0:.0f} s", flush=True)


def load(name: str) -> dict:
    """{index: expected output words} of a written set."""
    got = {}
    with open(path(name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x) for x in line.split()]
            got[v[0]] = np.array(v[1:], dtype=np.uint32)
    return got


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(SETS):
        make(nm)
