"""MI355X-native beam-plasma particle-in-cell step (arXiv:0808.4078 set-up).

The compute path is the HIP library ``libpic.so`` (sources in ``csrc/``,
C ABI in ``include/pic.h``); ``pic`` is its ctypes binding.  Build with
``python -m paper_0808_4078_amd.build``.
"""
from .pic import (PIC_FLAG_FREEZE_FIELDS, PIC_FLAG_HOST_LOAD, PIC_FLAG_LATTICE_LOAD,  # noqa: F401
                  PIC_FLAG_NO_COLLIDE, PIC_FLAG_NO_GRAPH, PIC_FLAG_TRACK_IDS, PIC_PREC_FP64,
                  PIC_PREC_MIXED, PicError, Run, lib, make_descs, query, workload_descs)
