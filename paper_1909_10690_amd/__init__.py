"""MI355X-native generalised-entropy mutual-information metric (arXiv 1909.10690).

``binding`` wraps the C-ABI library ``libgemi.so`` (hand-written HIP for
gfx950); ``inputs`` and ``transforms`` build seeded synthetic workloads.
The binding is imported lazily so that the input generators can be used on
machines without the built library.
"""

__all__ = ["binding", "inputs", "transforms"]


def __getattr__(name):
    if name == "binding":
        from . import binding
        return binding
    raise AttributeError(name)
