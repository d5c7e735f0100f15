"""Device ceilings beside the published peaks: the int8 matrix-core rate a
loop of random-operand MFMAs sustains (and with one operand's bytes 0 or 2,
as the shifted projection weights are), and the HBM read bandwidth of a plain
streaming kernel (``libhdc_ceilings.so``, built with the library).  Run as
``python -m paper_2606_26547_amd.ceilings``; bench.py --ceilings adds the
same figures to its record."""
from __future__ import annotations

import ctypes as C
import json
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhdc_ceilings.so")


def measure(reps: int = 5) -> dict:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhdc_ceilings.so is not built; run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    lib.hdc_ceiling_mfma_i8.restype = C.c_double
    lib.hdc_ceiling_mfma_i8.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.hdc_ceiling_mfma_i8_shifted.restype = C.c_double
    lib.hdc_ceiling_mfma_i8_shifted.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.hdc_ceiling_hbm_read.restype = C.c_double
    lib.hdc_ceiling_hbm_read.argtypes = [C.c_size_t, C.c_int, C.c_int]
    mfma = {"%d chains, %d wave/SIMD" % (c, w): lib.hdc_ceiling_mfma_i8(c, w, reps)
            for (c, w) in ((1, 1), (2, 1), (4, 1), (8, 1), (2, 2), (4, 2))}
    shifted = {"%d chains, %d wave/SIMD" % (c, w): lib.hdc_ceiling_mfma_i8_shifted(c, w, reps)
               for (c, w) in ((2, 1), (4, 1), (8, 1), (4, 2))}
    hbm = {"%d GiB, %d blocks/CU" % (g, b): lib.hdc_ceiling_hbm_read(g << 30, b, reps)
           for (g, b) in ((4, 4), (4, 8), (4, 16))}
    return {"mfma_i8_TOPs": mfma, "mfma_i8_shifted_TOPs": shifted, "mfma_i8_peak_TOPs": 5000.0,
            "hbm_read_GBs": hbm, "hbm_peak_GBs": 8000.0}


if __name__ == "__main__":
    print(json.dumps(measure(), indent=1))
