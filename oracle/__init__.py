"""CPU FP64 oracle for GLS estimation of SUR models -- TEST INFRASTRUCTURE.

This package is the slow, plainly-written reference that the HIP path is
checked against.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product package never does, and
nothing here imports the product package.  Inputs come from ``synth``.

Contents
  gls.py      closed-form / direct estimators (the definition of the result)
  pcg_aug.py  the PCG-Aug iteration in the paper's order and notation
              (FP64, and exact rational arithmetic for tiny integer data)
  grad.py     dense reference gradients of the GLS estimator (unrestricted
              and restricted)
  reduce.py   the SUR model reduction (QR of W = [X_1 ... X_G])
  pcg_ne.py   CG on the normal equations (the paper's PCG-NE comparator)

Parity status of every function is stated in its docstring.
"""
from . import gls, pcg_aug, pcg_ne, grad, reduce, mvrglm  # noqa: F401
