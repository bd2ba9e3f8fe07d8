"""Reader for the bracketed-block text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_blocks(name):
    blocks, key = {}, None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                key = line[1:-1]
                blocks[key] = []
            else:
                blocks[key].append([float(x) for x in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}
