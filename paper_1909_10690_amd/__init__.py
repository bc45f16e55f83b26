"""MI355X-native generalised-entropy mutual-information metric (arXiv 1909.10690).

Submodules: ``binding`` wraps the C-ABI library ``libgemi.so`` (hand-written
HIP for gfx950); ``autograd`` exposes the gradient as a torch autograd
Function; ``inputs`` and ``transforms`` build seeded synthetic workloads.
Nothing is imported eagerly, so the input generators work on machines
without the built library or a GPU.
"""
