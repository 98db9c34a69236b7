"""Compile the C oracle (test infrastructure) into oracle/_build/libigoracle.so.

``build`` makes the portable library the tests load (``-O3``, no CPU-specific
instructions: the library built here also runs on other hosts).  ``build_native``
makes a copy tuned for the host it runs on (``-O3 -march=native``); only the
benchmark's CPU-baseline leg uses it, built on the machine that times it.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ig_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libigoracle.so")
BASE_FLAGS = ["-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]


def _compile(out: str, extra) -> str:
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *BASE_FLAGS, *extra, "-o", tmp, SRC], check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    return _compile(LIB, [])


def build_native(out_dir: str) -> str:
    """The same source for this host's CPU (-march=native) into out_dir."""
    return _compile(os.path.join(out_dir, "libigoracle_native.so"), ["-march=native"])


if __name__ == "__main__":
    print(build())
