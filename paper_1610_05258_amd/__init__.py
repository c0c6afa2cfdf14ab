"""MI355X-native particle<->mesh assignment (Duque & Espanol, arXiv 1610.05258).

The compute path is the HIP library ``libp2m.so`` built from ``csrc/`` and
exposed through the C ABI declared in ``include/p2m.h``.  ``binding`` is a thin
ctypes layer over it (argument marshalling only); ``workloads`` generates the
seeded synthetic particle sets.  Importing the package loads nothing; the
library is opened on first use of ``binding`` and raises if it is missing.
"""
__all__ = ["binding", "workloads"]
