"""CPU oracle for the odd-even Kalman smoother -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
anything here; the GPU library never does, and this package imports nothing from
it.  Two independent references live here:

* ``dense``  -- the definition written out for tiny problems: the generalized
  least-squares estimate and (A^T W A)^{-1} of Sections II-A and IV, assembled as
  dense matrices (numpy);
* ``seq``    -- a plain sequential FP64 smoother in C (Paige-Saunders ordering
  plus Algorithm 1 of Section IV), usable at full size.
"""
