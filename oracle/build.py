"""Compile the CPU oracle with gcc (test infrastructure).

``build()`` writes oracle/liboracle.so, the copy the tests load: -O3 for the
generic x86-64 target, so that the same file runs on any host it is copied
to.  ``build(native=True, out=...)`` writes a copy tuned for the host that
compiles it (-O3 -march=native), which the benchmark's CPU-baseline leg
builds and times on the machine it runs on.  Both keep ISO C floating-point
semantics (no contraction into FMA, no fast-math), so they compute the same
values.  ``build(sanitize=True, out=...)`` adds AddressSanitizer and
UndefinedBehaviorSanitizer for the CPU sanitizer test.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(_HERE, "sscn_oracle.c"), os.path.join(_HERE, "sscn_sym_oracle.c")]
LIB = os.path.join(_HERE, "liboracle.so")


def build(verbose: bool = False, native: bool = False, sanitize: bool = False,
          out: str = LIB) -> str:
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O3", "-ffp-contract=off", "-fopenmp", "-fcx-fortran-rules",
           "-fPIC", "-shared", "-Wall", "-Wextra"]
    if native:
        cmd.append("-march=native")
    if sanitize:
        cmd += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=undefined"]
    cmd += ["-o", tmp] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
