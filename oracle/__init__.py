"""FP64 CPU oracle of the MUSCL-Hancock step, exact Riemann and Sedov-Taylor solutions.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product package.
"""
