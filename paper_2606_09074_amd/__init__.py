"""REFINE rendering-free importance scoring and pruning for MI355X (gfx950).

``api`` holds the Python front end of the C-ABI library ``librefine.so``
(``include/refine.h``); ``synth`` the seeded synthetic scenes; ``build``
compiles the HIP sources.
"""
