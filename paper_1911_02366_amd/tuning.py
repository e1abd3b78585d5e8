"""Persistent cache of the GEMM tile choice made by scdg_autotune.

The best tile configuration of the two batched GEMMs of the condensation
depends on the element problem sizes (n_i, n_c), the factor precision, the
device and the set of configurations the library offers.  A plan whose
signature is in the cache takes the stored choice without timing anything.
The cache is a JSON object {signature: entry}; it is rewritten atomically, and
an unreadable file counts as empty.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile
from collections import Counter

ENV_VAR = "SCDG_AUTOTUNE_CACHE"


def problem_signature(n_i, n_c, precision: str, device: str, configs) -> str:
    """Stable key of a plan's GEMM problems: the multiset of (n_i, n_c) pairs,
    the precision, the device name and the configuration list."""
    hist = sorted(Counter(zip((int(a) for a in n_i), (int(b) for b in n_c))).items())
    text = json.dumps({"sizes": hist, "precision": precision, "device": device, "configs": list(configs)},
                      sort_keys=True)
    return hashlib.sha256(text.encode()).hexdigest()[:24]


def default_path() -> str | None:
    return os.environ.get(ENV_VAR) or None


def load(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def lookup(path: str | None, key: str) -> dict | None:
    if not path:
        return None
    entry = load(path).get(key)
    if isinstance(entry, dict) and isinstance(entry.get("x"), str) and isinstance(entry.get("s"), str):
        return entry
    return None


def store(path: str | None, key: str, entry: dict) -> None:
    if not path:
        return
    data = load(path)
    data[key] = entry
    folder = os.path.dirname(os.path.abspath(path))
    os.makedirs(folder, exist_ok=True)
    fd, tmp = tempfile.mkstemp(prefix=".autotune", dir=folder)
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
