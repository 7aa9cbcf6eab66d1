"""MI355X (gfx950) separable-SOAP descriptor and GAP energy / forces.

Caro, "Optimizing many-body atomic descriptors for enhanced computational
performance of machine learning based interatomic potentials", arXiv:1905.02142.

The compute path is libsoap.so (hand-written HIP kernels behind the C ABI of
include/soap.h); this package only marshals torch tensors and streams into it.
"""
from . import _lib, autograd
from .soap import NeighbourList, Soap, SoapParams

__all__ = ["Soap", "SoapParams", "NeighbourList", "_lib", "autograd"]
