"""Build the C oracle with gcc (test infrastructure; see oracle/__init__.py).

``select_library(path)`` makes the loaders use another build of the same
sources (the sanitizer build of tests/sanitized_run.py); it must be called
before the first call into the oracle.
"""

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(_HERE, "nnm_oracle.c"), os.path.join(_HERE, "mesh_oracle.c")]
_LIB = os.path.join(_HERE, "libnnm_oracle.so")
_selected = None


def select_library(path) -> None:
    """Load the oracle from ``path`` (None: the default build)."""
    global _selected
    _selected = None if path is None else os.path.abspath(path)


def oracle_lib_path() -> str:
    return _selected or _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle sources into ``libnnm_oracle.so`` (always, when force)."""
    if _selected is not None:
        if not os.path.exists(_selected):
            raise FileNotFoundError(f"selected oracle build {_selected} does not exist")
        return _selected
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= max(os.path.getmtime(s) for s in SOURCES):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, *SOURCES, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB
