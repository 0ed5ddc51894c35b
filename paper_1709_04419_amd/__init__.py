"""H-matrix Gaussian log-likelihood on AMD MI355X (gfx950).

The product is the HIP library libhmlik.so behind the C ABI in
include/hmlik.h; `paper_1709_04419_amd.hmlik` is its Python binding and
`paper_1709_04419_amd.workloads` the seeded synthetic inputs.
"""
