"""FP64 CPU oracle for FDK and FDK-OD -- TEST INFRASTRUCTURE ONLY.

This package is the slow, plain reference that the GPU library is checked
against.  It is written from the paper "Fast optimal decomposed modification
of FDK with potential decreasing of memory consuming" (Andriiashen and
Kozhevnikov, 2017) and from the textbook FDK that the paper cites, in NumPy
float64, with no blocking, fusion or reordering beyond what the definitions
state.

Rules that keep it an independent checker:

* Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
  ``bench.py`` may import it.  The GPU product path never calls it, and it
  never imports anything from the GPU package.
* It shares no code with the HIP path: no kernels, helpers, tables or constant
  generators.  The seeded input generators live in ``synth/``, which holds
  none of the method's arithmetic.

Modules
-------
geometry   eq. (1) pix_pos, eq. (9) row position, angles, squares (Sec. 2.1/2.2)
fdk        cosine weight, Ram-Lak ramp filter, direct FDK backprojection
fdkod      bounds, crop + shift, angular decimation, folded backprojection
storage    FP16 / BF16 rounding emulation of stored sinograms
learned    learned decimation network (forward, backward, BP adjoint)
metrics    rel-RMSE, max-abs, sampled slices

Parity status of every function is stated in its docstring ("pinned by" lists
the independent facts the tests check it against).
"""

from . import geometry, fdk, fdkod, storage, metrics, learned  # noqa: F401
