#!/usr/bin/env python3
"""Write tests/golden/p256_requests.npz: seeded secp256r1 verification
requests whose signatures are made by the CPU oracle (keys d_i and nonces
from the seed, 32-byte random hashes, every 16th request corrupted), with the
oracle's verdicts.  The benchmark's serving workload reads this file, so it
needs no oracle code at run time.

    python tests/golden/make_p256_requests.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import c_oracle as co  # noqa: E402
from oracle import curves  # noqa: E402
from tests.common import seeded_signatures  # noqa: E402

M = 8192
SEED = 0x5E4E


def main() -> None:
    hashes, pubs, sigs = seeded_signatures(M, SEED)
    valid = co.ecdsa_verify(curves.SECP256R1.cid, hashes, pubs, sigs).astype(np.uint8)
    out = os.path.join(HERE, "p256_requests.npz")
    np.savez_compressed(out, hashes=hashes, pubkeys=pubs, sigs=sigs, valid=valid,
                        seed=np.array([SEED], dtype=np.uint64))
    print(f"wrote {out}: {M} requests, {int(valid.sum())} valid")


if __name__ == "__main__":
    main()
