"""MI355X-native LREI time stepping (arXiv 2508.21200): Python binding of liblrei.so."""
from .lrei import (Batch, Context, LreiError, Net, load, net_sample_floats, pair_entanglement,  # noqa: F401
                   MODELS, PAIRS, SCHEMES)
