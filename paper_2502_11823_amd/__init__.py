"""MI355X-native short-Fourier-transform inner products for long-duration
compact-binary gravitational-wave signals (Tenorio & Gerosa, arXiv:2502.11823).

The compute path is the HIP library ``libsft.so`` (C ABI declared in
``include/sft.h``); ``paper_2502_11823_amd.sft`` is its thin ctypes binding.
``paper_2502_11823_amd.synth`` draws seeded synthetic inputs.  Importing this
package loads nothing; the binding loads the library on first use and raises if
it is missing.
"""
__version__ = "0.1.0"
