"""Temporally parallel Kalman filter and RTS smoother for AMD MI355X (gfx950).

The scan elements and associative operators of Sarkka & Garcia-Fernandez,
"Temporal Parallelization of Bayesian Smoothers" (Lemmas 1-4), evaluated by
hand-written HIP kernels behind the C ABI declared in ``include/pks.h``.

``paper_1905_13002_amd.pks`` is the Python binding (ctypes, argument
marshalling only); importing it loads ``libpks.so`` and raises if the
library is missing.  ``paper_1905_13002_amd.workloads`` builds seeded
synthetic inputs and needs no GPU.
"""
__all__ = ["pks", "workloads"]
