"""MI355X-native hybrid lattice-Boltzmann / finite-difference Ericksen-Leslie step.

The compute path lives in the C-ABI library ``libel.so`` (hand-written HIP for
gfx950); ``paper_2503_06610_amd.el`` is its thin ctypes binding.  Importing the
package does not load the library, so the seeded-input module stays usable on
machines without a GPU.
"""
__all__ = ["el", "inputs"]
