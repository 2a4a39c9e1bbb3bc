"""FP64 CPU oracle of the DiskChunGS mapping-step hot path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constants) and imports
nothing from it; the only common input is the seeded generator module
``scenegen``.

The oracle is plain and slow on purpose.  Where the method reaches a result
that has a plain definition, the oracle computes that definition directly:

* hierarchical chunk culling   == a flat per-chunk exact box/frustum test
  (vertex enumeration of the intersection polytope)        -> ``chunks``
* compaction of active chunks  == concatenation in ascending EncodedID
* tile binning + radix sort    == for every pixel, all Gaussians whose pixel
  box contains it, in (float32 depth bits, index) order     -> ``splat``
* the hand-written adjoint      == reverse-mode derivative of the FP64
  forward definition (torch autograd on CPU, float64)      -> ``splat``
* Adam                          == the update written out   -> ``optim``

Parity status per function is stated in each module's header.  Every
function listed there is pinned by tests under ``tests/`` marked
``not gpu`` (closed forms, brute force, finite differences, library
routines), except where a header says "parity unpinned".
"""
