"""MI355X-native graph-neural-preconditioned FGMRES (Chen, ICLR 2025).

The compute path is the HIP library libgnp.so (C ABI in include/gnp.h); this
package only binds it.  Importing the package does not load the library;
``api`` does, and raises if it has not been built.
"""
__all__ = ["inputs"]
