"""MI355X (gfx950) native energy/force evaluation of an ANI-style neural
network potential (Deep-HP, arXiv 2207.14276): HIP kernels behind the C ABI
of include/nnp.h, with a thin ctypes binding and a torch.autograd.Function."""
from ._native import NNPError, load  # noqa: F401
from .model import NeighborPool, NNPFunction, NNPModel, Result  # noqa: F401
