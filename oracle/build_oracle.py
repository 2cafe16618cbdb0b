"""Build the oracle's C helper (liboracle_bins.so) with gcc.

Part of the test infrastructure; called by the repository's build entry point.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    src = os.path.join(HERE, "dft_bins.c")
    out = os.path.join(HERE, "liboracle_bins.so")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
    sys.exit(0)
