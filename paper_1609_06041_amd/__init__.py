"""MI355X-native FBP-preconditioned primal-dual TV reconstruction.

``paper_1609_06041_amd.ctpd`` is the Python binding of the HIP library
``libctpd.so`` (argument marshalling only); ``paper_1609_06041_amd.synth``
generates seeded synthetic phantoms and data.  Importing this package loads
neither.
"""
__all__ = ["ctpd", "synth"]
