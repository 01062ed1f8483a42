"""MI355X-native overlapping solution-transfer domain decomposition.

The hot path (transfer-block build, compression, interface GMRES with FP64
refinement, adjoint) lives in the HIP library ``libddst.so`` behind the C-ABI
of ``include/ddst.h``; ``ddst`` is its thin ctypes binding.  Importing this
package does not load the library; ``ddst.load_library()`` or the first
``Operator`` does, and fails loudly if it is missing.
"""
__all__ = ["ddst"]
