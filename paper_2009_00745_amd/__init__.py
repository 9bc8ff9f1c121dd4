"""MI355X (gfx950) TDSLDA time-step library: Python binding of liblise.so."""
from .lise import (Context, Batch, LiseError, load_library, version, coupling, SYMBOLS, LIB_PATH,
                   LISE_FP64, LISE_FP32, LISE_FP32_MFMA)
