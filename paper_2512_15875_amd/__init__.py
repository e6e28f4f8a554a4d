"""MI355X (gfx950) hot path of the TTNS/TTNO vibrational eigensolver of
arXiv 2512.15875: environment updates and block H_eff products on the CDNA4
matrix cores, behind the C ABI of include/ttn.h (libttn.so)."""
from . import ttn  # noqa: F401
