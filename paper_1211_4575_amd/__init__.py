"""MI355X-native particle step of the Photon-Plasma relativistic PIC method (arXiv:1211.4575).

The compute path is the HIP library ``libpp.so`` behind the C ABI declared in
``include/pp.h``; :mod:`paper_1211_4575_amd.pp` is its thin ctypes binding.
Importing the package loads nothing; the binding loads the library on first use
and raises if it is missing.
"""
