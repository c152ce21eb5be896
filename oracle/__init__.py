"""CPU oracle: test infrastructure only.

Plain FP64 CPU implementation of the mixed-variational band-structure method,
an independent displacement plane-wave expansion, the 1-D transfer-matrix
dispersion relation and the error metric.  Only the tests, the smoke check and
the benchmark's CPU-baseline leg import it; the product path never does.
"""
