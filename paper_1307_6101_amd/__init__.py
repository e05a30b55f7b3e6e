"""MI355X (gfx950) implementation of the DD-alpha-AMG solver hot path
(Frommer, Kahl, Krieg, Leder, Rottmann, arXiv:1307.6101).

The product is the C-ABI library ``libddamg.so`` (include/ddamg.h), built
from ``csrc/`` by ``build.py``; ``ddamg`` is its thin Python binding.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddamg.so")
