"""MI355X-native recursive differentiable transparent-mesh ray tracer.

The compute path lives in the HIP library ``libdifftrans.so`` (sources in
``csrc/``, C-ABI in ``include/difftrans.h``); ``binding`` marshals arguments
to it with ctypes.  Importing this package loads nothing: the library is
opened on first use and a missing library raises immediately.
"""
__all__ = ["synth"]
