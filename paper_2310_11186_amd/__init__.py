"""MI355X-native t-SGNE optimisation loop (Li, Xiao, Zhou, arXiv 2310.11186).

The compute path is the HIP library ``libtsgne.so`` (C-ABI, declared in
``include/tsgne.h``); :mod:`paper_2310_11186_amd.tsgne` is its thin ctypes
binding and :mod:`paper_2310_11186_amd.synth` draws seeded synthetic inputs.
"""
__all__ = ["tsgne", "synth"]
