"""MI355X-native hybrid ocean hot path (FFT background + frequency-bucketed
wave particles), after Xue et al., arXiv 2511.02852.

The compute path lives in the HIP library built from ``csrc/`` (C ABI in
``include/hwo.h``); :mod:`paper_2511_02852_amd.hwo` is a thin ctypes binding
and :mod:`paper_2511_02852_amd.scenes` draws seeded synthetic inputs.
"""
