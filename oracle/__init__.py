"""FP64 CPU oracles of the gliding-assay micro-step.  TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's CPU-baseline leg may import
this package.  Two independent implementations of the same scheme live here:

* `oracle_a` - plain C99 loops (liboracle.so), FP64, OpenMP over x rows.  The reference
  for every forward parity check and the CPU timing baseline.
* `oracle_torch` - plain PyTorch CPU float64 tensor ops, written separately; its autograd
  gives the FP64 reference adjoint.

Neither shares code with the HIP path (no kernels, headers, tables or helpers).
"""
