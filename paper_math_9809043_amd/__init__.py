"""Recursive multi-scale preconditioned conjugate gradient for -div(K grad p) = f on MI355X.

`paper_math_9809043_amd.mscg` is the binding of the HIP library (libmscg.so);
`paper_math_9809043_amd.synth` draws the seeded synthetic workloads.  Importing
the package does not load the library; the first call that needs the GPU does,
and raises if it has not been built.
"""
