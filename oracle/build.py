"""Compile the CPU oracle (test infrastructure) into oracle/libohm_oracle.so."""
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libohm_oracle.so")
SRC = [os.path.join(HERE, "ohm_oracle.c")]


def source_digest() -> str:
    """sha256 of the oracle's source, embedded by the build (orc_source_digest)."""
    h = hashlib.sha256()
    for f in SRC:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
           f'-DORC_SOURCE_DIGEST="{source_digest()}"', *SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
