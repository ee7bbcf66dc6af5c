"""MI355X-native coupled electrokinetic lattice step (arXiv:1712.08494).

The compute path lives in the HIP library ``libek.so`` behind the C ABI in
``include/ek.h``; ``paper_1712_08494_amd.ek`` is its Python binding.  Importing the
package does not load the library, so CPU-only code (input generation) works without it.
"""
