"""Measured issue rates of the gfx950 units the resultant kernels use.

``measure()`` runs the microbenchmarks of ``csrc/peak.hip`` (libpeak.so, built
by ``build.py``) on one device: eight independent dependency chains per lane,
four waves on every SIMD, timed with HIP events.  The rates are what the
roofline of the evaluation stage is also reported against (beside the peak
derived from unit counts and clock): the vector ALU part against the fused
three-product update and the Montgomery product, the matrix-core part against
the int8 matrix product.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
KINDS = {0: "v_add_u32", 1: "v_mul_lo_u32", 2: "mad_u64_u32", 3: "montgomery_mul", 4: "fused_update_3_products",
         5: "mfma_i32_16x16x32_i8_macs"}


def _lib():
    path = os.path.join(_PKG, "libpeak.so")
    if not os.path.exists(path):
        raise RuntimeError("libpeak.so is not built (run paper_1010_1386_amd.build)")
    lib = ctypes.CDLL(path)
    lib.rsl_peak_rate.restype = ctypes.c_int
    lib.rsl_peak_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    return lib


def measure(device=0, waves=(4, 8), iters=4096, reps=5):
    """Rates in operations per second (lane operations; MACs for the matrix
    kind), the best over the given waves per SIMD."""
    import torch

    props = torch.cuda.get_device_properties(device)
    cus = props.multi_processor_count
    lib = _lib()
    sink = torch.zeros(cus * 4 * max(waves) * 64, dtype=torch.int32, device=f"cuda:{device}")
    torch.cuda.synchronize(device)
    out = {"cus": cus, "waves_per_simd": list(waves), "chains_per_lane": 8}
    for kind, name in KINDS.items():
        best = 0.0
        for w in waves:
            r = ctypes.c_double()
            it = iters if kind != 5 else max(1, iters // 8)
            rc = lib.rsl_peak_rate(device, kind, cus, w, it, reps, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(r))
            if rc:
                raise RuntimeError(f"rsl_peak_rate({name}) failed: {rc}")
            best = max(best, r.value)
        out[name] = best
    return out


if __name__ == "__main__":
    import json

    print(json.dumps(measure()))
