"""Writes datagen_sha256.txt: SHA-256 of fixed outputs of the seeded generators.

Run from the repository root: python -m tests.golden.make_datagen_digests
It calls only the input generators (no matching code).
"""
import hashlib
import os

import datagen as dg


def digests() -> dict:
    out = {}
    out["uniform_n2^20_sigma4_seed1"] = dg.uniform_text(1 << 20, 4, seed=1)
    out["uniform_n2^20_sigma256_seed1"] = dg.uniform_text(1 << 20, 256, seed=1)
    out["zipf_n2^20_K64_s1.0_seed1"] = dg.zipf_text(1 << 20, 64, 1.0, seed=1)
    out["lengths_4096_2_1024_seed3"] = dg.log_uniform_lengths(4096, 2, 1024, seed=3)
    return {k: hashlib.sha256(v.tobytes()).hexdigest() for k, v in out.items()}


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "datagen_sha256.txt")
    with open(path, "w") as f:
        f.write("# written by tests/golden/make_datagen_digests.py\n")
        for k, v in digests().items():
            f.write("%s %s\n" % (k, v))
    print(open(path).read())
