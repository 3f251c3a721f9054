"""MI355X-native split pressure-gradient projection step (arXiv 2103.01874, Sec. 5.4).

The compute path is the HIP library ``libppe.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/ppe.h``; ``binding`` marshals torch tensors to
it.  Importing this package does not load the library; ``binding.load()`` does,
and fails loudly when it has not been built.
"""

__all__ = ["binding", "synth", "serve"]
