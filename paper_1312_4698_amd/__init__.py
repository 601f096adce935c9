"""MI355X-native TA-SC-IVR power spectra (time-averaged semiclassical initial
value representation with the separable prefactor approximation).

The compute path is the HIP library ``libscivr.so`` behind the C ABI declared
in ``include/scivr.h``; :mod:`paper_1312_4698_amd.scivr` is its thin binding.
:mod:`paper_1312_4698_amd.inputs` builds the synthetic problem definitions.
Importing the package does not load the library.
"""

__all__ = ["inputs", "scivr"]
