"""MI355X-native optimized Schwarz solver for the 2-D NLS / GPE
(Besse & Xing, arXiv:1603.05110): HIP kernels behind the C ABI of
include/osm.h, with a thin ctypes binding in `osm`."""
