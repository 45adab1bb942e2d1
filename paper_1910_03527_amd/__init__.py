"""MI355X-native generalized MBE-FCI hot path (arXiv:1910.03527).

Thin Python binding over the C ABI of ``include/mbefci.h`` (library
``libmbefci.so``, hand-written HIP for gfx950).  PyTorch supplies device
memory and streams; every step of the computation runs in the library's
kernels, and the binding only marshals arguments.

Names mirror the C ABI without the ``mbefci_`` prefix:

* ``Context``            -- mbefci_create / mbefci_destroy / options
* ``num_strings``, ``num_links``, ``num_tuples``
* ``strings``, ``link_table``                  (host string / link tables, no context)
* ``Context.strings``, ``Context.link_table``  (the same tables built on the device)
* ``Context.hdiag``, ``Context.sigma``, ``Context.sigma_noalloc``  (one CASCI Hamiltonian)
* ``Context.casci``                            (mbefci_casci_batch: same-shape CASCIs)
* ``Context.casci_one``, ``casci``             (mbefci_casci: one CASCI, its CI vector and RDMs)
* ``Context.casci_rdm``                        (RDMs of the last CASCI solve)
* ``sym_ndet``, ``Context.casci_sym``, ``Context.sigma_sym``  (point-group blocked CASCIs)
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
    link_table,
    MBEEnergy,
    num_links,
    num_strings,
    num_tuples,
    partition,
    strings,
    sym_ndet,
    TYPE1,
    TYPE2,
    TYPE3,
)
