"""MI355X (gfx950) implementation of the per-iteration hot path of particle-based
Region Competition with particle-approximated Sobolev gradients
(Sbalzarini, Schneider, Cardinale, arXiv:1403.0240).

``sobrc`` is the Python binding of the C ABI (include/sobrc.h);
``workloads`` builds seeded synthetic inputs.
"""
