"""MI355X-native finite-element (unlumped mass-matrix) Maxwell field step.

Importing the package does not load the HIP library; ``paper_1907_13088_amd.mx``
loads it on first use and raises if it has not been built.
"""
__all__ = ["inputs", "mx"]
