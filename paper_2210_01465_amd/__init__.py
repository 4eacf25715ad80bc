"""MI355X-native engine for the fitness-flow-graph landscape metric.

``synth`` (seeded synthetic search spaces) imports without torch or a GPU.
The engine itself is the C-ABI library ``libfl.so`` (HIP, gfx950); its Python
binding is ``api`` and is imported on first use.
"""
__all__ = ["api", "synth", "build"]


def __getattr__(name):
    if name in ("api", "synth", "build", "_abi"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
