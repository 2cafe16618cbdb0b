"""Build the oracle's C helpers (liboracle_bins.so: per-bin sums and the
whole-vector per-target form) with gcc.

Part of the test infrastructure; called by the repository's build entry point.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    srcs = [os.path.join(HERE, f) for f in ("dft_bins.c", "qft_state.c")]
    out = os.path.join(HERE, "liboracle_bins.so")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared"] + srcs + ["-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
    sys.exit(0)
