"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Compile bss_oracle.c and bss_oracle8.c with gcc (no fast-math: the oracle must follow IEEE double)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-o", LIB + ".tmp", os.path.join(HERE, "bss_oracle.c"),
           os.path.join(HERE, "bss_oracle8.c"), "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
