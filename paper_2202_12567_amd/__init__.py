"""MI355X-native sparse sampling and completion of VPL lighting matrices
(Huo, Wang, Liu, Bao, arXiv 2202.12567): HIP kernels for gfx950 behind the
C ABI of include/vplmc.h, with a thin Python binding in ``api``."""
