"""MI355X-native differentiable two-point-correlation descriptor (arXiv 2103.09686).

The compute path lives in the HIP library ``libdmcr.so`` (sources under
``csrc/``, C ABI in ``include/dmcr.h``).  Importing this package loads
nothing; the binding in ``dmcr`` loads the library on first use and raises
if it is missing -- there is no CPU fallback.
"""

__all__ = ["dmcr", "synth"]
