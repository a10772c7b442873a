"""Build the C oracle with gcc (test infrastructure; see oracle/__init__.py)."""

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "nnm_oracle.c"), os.path.join(_HERE, "mesh_oracle.c")]
_LIB = os.path.join(_HERE, "libnnm_oracle.so")


def oracle_lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle sources into ``libnnm_oracle.so`` (always, when force)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= max(os.path.getmtime(s) for s in _SRCS):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, *_SRCS, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB
