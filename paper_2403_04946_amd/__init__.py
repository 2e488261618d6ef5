"""MI355X tensor-train solver for the Burgers-Hopf characteristic-function PDE.

The compute path is the HIP shared library ``libttfde.so`` (C ABI declared in
``include/tt_fde.h``); ``paper_2403_04946_amd.tt`` is a thin ctypes binding
with the same entry-point names.  Importing this package does not load the
library; ``paper_2403_04946_amd.tt.lib()`` does, and raises if it is missing.
"""
