"""Persistent autotune cache (JSON) for the batched registration plan.

The batched path times its eight plans (split length x E-step tile) on the
first two iterations of a batch.  The choice depends on the device and on the
shape of the batch, so it is stored in a JSON file keyed by
(arch, kernel, M bucket, N bucket, D, precision, instance-count bucket), where
a bucket is ceil(log2(n)) of the batch's mean set size (or of the instance
count).  A later batch with the same key forces the stored plan untimed.

Host logic only: nothing here touches device memory or the library.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
import warnings

VERSION = 1


def bucket(n: float) -> int:
    """ceil(log2(n)) for n >= 1 (0 for n <= 1)."""
    return 0 if n <= 1 else int(math.ceil(math.log2(n)))


def make_key(arch: str, kernel: str, M: float, N: float, D: int, precision: str,
             count: int = 1) -> str:
    return (f"{arch}|{kernel}|M{bucket(M)}|N{bucket(N)}|D{int(D)}|{precision}"
            f"|B{bucket(count)}")


def batch_key(arch: str, Ms, Ns, D: int = 3, precision: str = "fp32") -> str:
    """Key of a batch of registrations with set sizes Ms[i] x Ns[i]."""
    if len(Ms) == 0 or len(Ms) != len(Ns):
        raise ValueError("batch_key needs one M and one N per instance")
    return make_key(arch, "batch", sum(Ms) / len(Ms), sum(Ns) / len(Ns), D, precision,
                    len(Ms))


class TuneCache:
    """A JSON file {key: entry}; entries are plain dicts.  Writes replace the
    file atomically (write to a temporary file in the same folder, then
    rename), so a reader never sees a partial file; a file that does not
    parse, or has another version, is treated as empty (with a warning) and
    rewritten on the next put."""

    def __init__(self, path: str):
        self.path = os.path.abspath(path)

    def _load(self) -> dict:
        try:
            with open(self.path) as f:
                data = json.load(f)
        except FileNotFoundError:
            return {}
        except (OSError, ValueError) as e:
            warnings.warn(f"tune cache {self.path} unreadable ({e}); ignoring it")
            return {}
        if not isinstance(data, dict) or data.get("version") != VERSION \
                or not isinstance(data.get("entries"), dict):
            warnings.warn(f"tune cache {self.path} has another format; ignoring it")
            return {}
        return data["entries"]

    def get(self, key: str):
        e = self._load().get(key)
        return dict(e) if isinstance(e, dict) else None

    def put(self, key: str, entry: dict) -> None:
        entries = self._load()
        entries[key] = dict(entry)
        d = os.path.dirname(self.path)
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(prefix=".tune_", suffix=".json", dir=d)
        try:
            with os.fdopen(fd, "w") as f:
                json.dump({"version": VERSION, "entries": entries}, f, indent=1,
                          sort_keys=True)
            os.replace(tmp, self.path)
        except BaseException:
            if os.path.exists(tmp):
                os.unlink(tmp)
            raise

    def __len__(self):
        return len(self._load())
