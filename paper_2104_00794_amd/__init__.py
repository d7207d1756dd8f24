"""MI355X-native probed adjoint-state FWI gradients (Louboutin & Herrmann,
"Ultra-low memory seismic inversion with randomized trace estimation").

The compute path is the HIP library ``libtpx.so`` (C-ABI, ``include/tpx.h``);
``paper_2104_00794_amd.tpx`` is its thin ctypes binding.  Importing this
package loads nothing; the binding loads the library on first use and raises if
it is missing.
"""
__all__ = ["inputs", "tpx"]
