"""MI355X-native hot path of block RRQR filtering + right-preconditioned LSQR for ELM-FBPINNs.

Importing the package loads nothing native; ``paper_2506_17626_amd.rfm`` is the
binding to the HIP library (it raises if the library is missing) and
``paper_2506_17626_amd.instances`` draws the seeded synthetic inputs.
"""
__all__ = ["instances", "rfm"]
