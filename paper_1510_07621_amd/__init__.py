"""MI355X-native P3M periodic-gravity force (CONCEPT, arXiv:1510.07621).

The force path lives in the HIP library ``libp3m.so`` (sources under
``csrc/``, C-ABI declared in ``include/p3m.h``). ``binding`` exposes the same
entry points to Python with PyTorch tensors for device memory and streams;
``ics`` draws the seeded synthetic particle sets. Importing the package does
not load the library; ``binding`` does, and raises if it is not built.
"""
__all__ = ["ics", "binding"]
