"""Python wrapper of the request server (rsl_server_* in include/rsl.h)."""

from __future__ import annotations

import ctypes

from . import (RSLError, RSL_EAGAIN, _Result, _as_poly, _lib, _var_code, _vp, rsl_info, rsl_stats)

RSL_ETIMEDOUT = -7


class Server:
    """Continuous-batching request server on a Context.

    submit() copies the inputs and returns a ticket; wait(ticket) returns the
    resultant (list of ints).  Admission is FIFO by slots and device footprint.
    """

    def __init__(self, ctx, budget_bytes=64 << 20, max_slots=64, max_queue=4096):
        self.ctx = ctx
        ctx._owned.add(self)
        h = _vp()
        rc = _lib.rsl_server_create(ctx.h, budget_bytes, max_slots, max_queue, ctypes.byref(h))
        if rc:
            raise RSLError(rc, "rsl_server_create: " + ctx.last_error())
        self.h = h
        self._outs = {}

    def plan(self, f, g, var="y"):
        """Plan a request without queueing it: (handle, result buffer) for enqueue()."""
        pf, pg = _as_poly(f), _as_poly(g)
        # planned once in the library: the plan sizes the result buffer and the
        # scheduler lays the request's batch out from the same plan
        info = rsl_info()
        handle = ctypes.c_uint64()
        rc = _lib.rsl_server_plan(self.h, ctypes.byref(pf.c), ctypes.byref(pg.c), _var_code(var),
                                  ctypes.byref(info), ctypes.byref(handle))
        if rc:
            raise RSLError(rc, "rsl_server_plan: " + self.ctx.last_error())
        return handle.value, _Result(max(info.D, 0), info.out_limbs)

    def enqueue(self, planned):
        """Queue a planned request; the ticket (RSLError RSL_EAGAIN when the queue is full)."""
        handle, out = planned
        t = ctypes.c_uint64()
        rc = _lib.rsl_server_enqueue(self.h, handle, ctypes.byref(out.c), ctypes.byref(t))
        if rc:
            raise RSLError(rc, "rsl_server_enqueue")
        self._outs[t.value] = out
        return t.value

    def submit(self, f, g, var="y"):
        return self.enqueue(self.plan(f, g, var))

    def try_submit(self, f, g, var="y"):
        """Like submit() but returns None when the server queue is full."""
        try:
            return self.submit(f, g, var)
        except RSLError as e:
            if e.code == RSL_EAGAIN:
                return None
            raise

    def poll(self, ticket):
        st = ctypes.c_int()
        rc = _lib.rsl_server_poll(self.h, ticket, ctypes.byref(st))
        if rc < 0:
            raise RSLError(rc, "rsl_server_poll")
        if rc == 0:
            return None
        out = self._outs.pop(ticket)
        if st.value:
            raise RSLError(st.value, "request failed")
        return out.value()

    def wait(self, ticket, timeout_ms=-1, raw=False):
        """The resultant as a list of ints, or with raw=True its limb buffer (a
        result object: .deg, .c.limbs, .raw()) without the conversion to ints."""
        rc = _lib.rsl_server_wait(self.h, ticket, timeout_ms)
        if rc == RSL_ETIMEDOUT:
            return None
        out = self._outs.pop(ticket)
        if rc:
            raise RSLError(rc, "request failed")
        return out if raw else out.value()

    def stats(self):
        s = rsl_stats()
        _lib.rsl_server_stats(self.h, ctypes.byref(s))
        return {name: getattr(s, name) for name, _ in rsl_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            _lib.rsl_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
