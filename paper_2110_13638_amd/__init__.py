"""MI355X-native RNS-CKKS ciphertext arithmetic for encrypted neural-network
inference (EDLaaS, arXiv 2110.13638): hand-written gfx950 kernels behind the
C ABI of ``libckks_hip.so`` (declared in ``include/ckks.h``), a thin ctypes
binding (``_native``), device-resident objects (``ckks``), the graph
runtime of the paper's Algorithms 1-5 (``graph``), network lowerings
(``nets``) and a continuous-batching server (``serve``)."""
