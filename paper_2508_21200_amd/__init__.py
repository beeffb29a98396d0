"""MI355X-native LREI time stepping (arXiv 2508.21200): Python binding of liblrei.so."""
from .lrei import Batch, Context, LreiError, load, MODELS, SCHEMES  # noqa: F401
