"""MI355X-native 2.5D axisymmetric PIC step (PICsar, arXiv 1407.1810).

The product path is the HIP library ``libpicsar_hip.so`` behind the C ABI in
``include/picsar_hip.h``; ``binding`` marshals arguments to it.  Importing the
package does not load the library; ``binding.Sim`` does, and fails loudly if
it has not been built.
"""
__version__ = "0.1.0"
