"""Per-stage kernel timing through librpt's HIP events (see rpt_timing_* in rpt.h)."""
from __future__ import annotations

import ctypes as C

from . import _lib


def enable(on: bool = True) -> None:
    _lib.load().rpt_timing_enable(1 if on else 0)


def reset() -> None:
    _lib.load().rpt_timing_reset()


def stages() -> list[str]:
    lib = _lib.load()
    buf = C.create_string_buffer(4096)
    lib.rpt_timing_stages(buf, 4096)
    s = buf.value.decode()
    return [x for x in s.split(",") if x]


def query(stage: str):
    """(total_ms, launches) of one stage, or None if it has no records."""
    lib = _lib.load()
    ms = C.c_double(0.0)
    cnt = C.c_int64(0)
    rc = lib.rpt_timing_query(stage.encode(), C.byref(ms), C.byref(cnt))
    if rc != 0:
        return None
    return ms.value, int(cnt.value)


def summary() -> dict:
    return {s: query(s) for s in stages()}
