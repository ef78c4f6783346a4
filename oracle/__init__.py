"""FP64 CPU oracle of the Photon-Plasma particle step (arXiv:1211.4575).

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never does.
"""
