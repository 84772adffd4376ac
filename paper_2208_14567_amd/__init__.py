"""MI355X-native batched simulation of 1-DOF planar linkages (LINKS hot path).

Submodules are imported lazily: ``gen`` (seeded inputs) needs only numpy, while
``links`` loads the HIP library ``liblinks.so`` and fails loudly without it.
"""
__all__ = ["gen", "links"]
