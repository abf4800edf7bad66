"""GAME fitness evaluation and genetic step on AMD Instinct MI355X (gfx950).

The compute path is the HIP shared library ``libgame.so`` built from
``csrc/``; ``paper_1304_0597_amd.game`` is a thin ctypes binding to its C ABI
(``include/game.h``).  ``datagen`` holds the seeded synthetic workloads.
Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
