"""MI355X-native FMM for the 3-D Laplace equation in layered media (arXiv:1908.10863).

Importing the package loads nothing; ``paper_1908_10863_amd.fmmlm`` binds the
HIP library and fails loudly when it is missing.
"""
