"""MI355X-native geometric multigrid for the H(div)-DG Brinkman/Darcy equations.

The HIP library (libbmg.so, C ABI in include/bmg.h) is loaded by the `bmg`
submodule; `inputs` holds the seeded synthetic input generators.
"""
