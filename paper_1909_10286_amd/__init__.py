"""MI355X-native batched candidate evaluator for the GPU heuristic search of
multi-tour biomass logistics (Plessen, arXiv 1909.10286).

Submodules: ``inputs`` (seeded synthetic instances), ``bl`` (ctypes binding of
the HIP library libbl.so), ``build`` (hipcc build of the library).  Importing
the package loads nothing; ``bl.load()`` loads the library.
"""
