"""FP64 CPU oracle of the quasi-Monte Carlo radiative-transfer path.

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU library is checked
against.  Only tests/, the smoke check and the benchmark's CPU-baseline leg may
import it; the product never does, and it imports nothing from the product.
"""
