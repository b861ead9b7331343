"""MI355X-native batched affine-gap seed extension (SALoBa, arXiv 2301.09310).

The compute path is the HIP library ``libsalo.so`` built from ``csrc/``;
``paper_2301_09310_amd.salo`` is its thin ctypes binding.  Importing this
package does not load the library; ``inputs`` draws the synthetic workloads.
"""
__all__ = ["inputs", "salo"]
