"""MI355X (gfx950) relaxation step of the multi-phase SPH mesh generator of Ji, Fu, Hu &
Adams (arXiv 1906.07925): HIP kernels behind the C ABI of ``include/mpsph.h``."""

__all__ = ["mpsph", "workloads"]
