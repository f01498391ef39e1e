"""MI355X-native Grangeat / epipolar-consistency engine (arxiv 1806.02637).

``binding`` is the ctypes layer over ``libecc.so`` (the C ABI of
``include/ecc.h``); ``engine`` wraps it with torch device tensors;
``autograd`` exposes the cost as a ``torch.autograd.Function``; ``serve`` is
the continuous-batching server; ``inputs`` generates seeded synthetic scans.
Importing the package loads nothing: the library is opened on first use.
"""
__all__ = ["binding", "engine", "autograd", "serve", "inputs"]
