"""MI355X-native generalized MBE-FCI hot path (arXiv:1910.03527).

Thin Python binding over the C ABI of ``include/mbefci.h`` (library
``libmbefci.so``, hand-written HIP for gfx950).  PyTorch supplies device
memory and streams; every step of the computation runs in the library's
kernels, and the binding only marshals arguments.

Names mirror the C ABI without the ``mbefci_`` prefix:

* ``Context``            -- mbefci_create / mbefci_destroy / options
* ``num_strings``, ``num_links``, ``num_tuples``
* ``Context.strings``, ``Context.link_table``  (device string / link tables)
* ``Context.hdiag``, ``Context.sigma``         (one CASCI Hamiltonian)
* ``Context.casci``                            (batch of same-shape CASCIs)
* ``casci``                                    (one CASCI, optionally with its RDMs)
* ``Context.casci_rdm``                        (their 1- and 2-RDMs)
* ``Context.mbe_forward``, ``Context.mbe_backward``  (Eq. 1 / Eq. 2)
* ``Context.mbe_screened``  (order-by-order expansion with the Eq. 4 screening)
* ``partition``  (the Type-1/2/3 reference/expansion partitions)
* ``MBEEnergy``  -- ``torch.autograd.Function`` over forward/backward.
"""
from __future__ import annotations

from .binding import (  # noqa: F401
    BATCHED,
    PER_LAUNCH,
    Context,
    MbefciError,
    casci,
    MBEEnergy,
    num_links,
    num_strings,
    num_tuples,
    partition,
    TYPE1,
    TYPE2,
    TYPE3,
)
