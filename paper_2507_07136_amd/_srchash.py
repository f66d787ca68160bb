"""Fingerprint of the library's sources (csrc/*.hip, csrc/*.h and
include/ls2.h): baked into libls2.so at build time and compared when the
binding loads it, so a library built from other sources is never used."""
from __future__ import annotations

import glob
import hashlib
import os

_HERE = os.path.dirname(os.path.abspath(__file__))


def source_files():
    csrc = os.path.join(_HERE, "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h")))
    return files + [os.path.join(os.path.dirname(_HERE), "include", "ls2.h")]


def source_hash():
    """sha256 prefix over the sources' names and bytes; None when they are
    not present."""
    files = source_files()
    if not all(os.path.exists(f) for f in files):
        return None
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
