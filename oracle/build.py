"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so,
and its operation-census variant (the same sources with ORC_CENSUS defined,
whose counters oracle/census.py reads) into oracle/liboracle_census.so.

Plain gcc; no GPU code and nothing shared with the HIP library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["faddeeva.c", "me_forward.c", "lm.c"]
LIB = os.path.join(HERE, "liboracle.so")
CENSUS_LIB = os.path.join(HERE, "liboracle_census.so")


def _gcc(out, defines, verbose):
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = (["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-Wall", "-Wextra",
            "-Wno-unused-parameter", "-fno-fast-math", "-ffp-contract=off"]
           + ["-D" + d for d in defines] + ["-o", tmp] + srcs + ["-lm", "-lpthread"])
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    return _gcc(LIB, [], verbose)


def build_census(verbose: bool = False) -> str:
    return _gcc(CENSUS_LIB, ["ORC_CENSUS"], verbose)


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_census(verbose=True))
