"""MI355X-native implicit chemical-kinetics update (Le & Cambier, arXiv:1110.4903).

Submodules:
  synth  -- seeded synthetic mechanisms and cell states (input generation only)
  kin    -- ctypes binding of the C-ABI library libkin.so (argument marshalling only)
  serve  -- continuous-batching request loop over the binding

Importing the package imports nothing else; the HIP library is loaded on first use
of ``paper_1110_4903_amd.kin``.
"""

__version__ = "0.1.0"
