"""CPU baseline B of the benchmark: the oracle's BKS algorithm with its three
tensor-times-block contractions replaced by C++/OpenMP FP64 kernels
(ttmc_omp.cpp) on all host cores, and numpy's BLAS/LAPACK threads on all
cores for the dense steps.  A measurement baseline only: checked against the
FP64 oracle by the CPU tests, timed by bench.py's cpu_baseline leg; the GPU
library never uses it."""
