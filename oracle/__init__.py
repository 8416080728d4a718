"""Plain FP64 CPU oracle for HOTRG — TEST INFRASTRUCTURE, not part of the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The GPU path
(``paper_2602_05900_amd``) never imports it and shares no code with it.

Modules
-------
``hotrg``  the HOTRG coarse-graining algorithm, step by step, in NumPy FP64
           (Sec. II.A, Eq. (2) of the paper; the algorithm it cites, Xie et al.,
           Phys. Rev. B 86, 045139 (2012)).
``exact``  independent pins: brute-force spin sums, spin and tensor transfer
           matrices, Onsager's exact solution.
``itebd``  imaginary-time evolution of an infinite two-site chain (Sec. II.A,
           Eq. (1); the iTEBD algorithm it cites, Vidal, PRL 98, 070201
           (2007), in Hastings' inverse-free update), NumPy FP64.
"""
