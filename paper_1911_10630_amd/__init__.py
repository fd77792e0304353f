"""MI355X-native localized-orbital exact exchange (pair Poisson hot path).

Submodules are imported lazily: ``synth`` (seeded inputs) never loads the
HIP library; ``exx`` (the binding) does.
"""
__all__ = ["synth", "exx"]
