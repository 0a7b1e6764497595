"""Compile the C oracle (test infrastructure) into oracle/liboracle.so with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def library_path():
    return os.path.join(HERE, "liboracle.so")


def build():
    src = os.path.join(HERE, "oracle.c")
    out = library_path()
    tmp = out + ".tmp"
    # plain IEEE arithmetic: no -ffast-math, no FMA contraction
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
