"""FP64 CPU oracle of the Horseshoe Probit Gibbs sweep.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.
"""
