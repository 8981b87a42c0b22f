"""MI355X particle advance of the non-hybrid joint velocity-frequency-scalar
PDF method (Bakosi, Franzese & Boybeyi, arXiv:1006.0549).

The computation lives in the HIP library libpdfmc.so (C ABI: include/pdfmc.h);
`pdfmc.Sim` is its Python binding.
"""
from .pdfmc import Sim, PdfmcError, lib, LIB_PATH, EXPORTS, COUNTER_NAMES, NF  # noqa: F401
