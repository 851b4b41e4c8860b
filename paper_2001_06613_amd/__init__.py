"""MI355X-native spatio-temporal multilevel registration (arXiv 2001.06613).

The registration path runs in the HIP library ``libstml.so`` built from
``csrc/``; ``binding`` wraps its C-ABI (declared in ``include/stml.h``).
``synth`` draws the seeded synthetic sequences.
"""
