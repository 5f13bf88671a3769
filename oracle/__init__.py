"""CPU oracle of the sampled-trial AFQMC step (FP64 / complex128, numpy).

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the CPU-baseline
leg of the benchmark import this package.  The product (the HIP library and
its Python binding) never imports it, and it never imports the product.
"""
