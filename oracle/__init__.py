"""CPU oracle (test infrastructure only).

A plain, slow FP64 NumPy implementation of the implicit difference scheme
(IDS) of Gu, Huang, Ji, Carpentieri and Alikhanov (arXiv:1603.00279) for the
time-space fractional convection-diffusion equation.  It is used only by the
tests, by ``__graft_entry__.smoke()`` and by the CPU-baseline leg of
``bench.py``; the product path never imports it.  It shares no code with the
HIP path: the only common inputs come from the ``workloads`` package.
"""
from .ids_oracle import *  # noqa: F401,F403
