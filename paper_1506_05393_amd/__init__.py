"""libmrf: MRF dictionary generating and searching on MI355X (gfx950).

The compute path is the HIP library libmrf.so (built in-tree); this package
is its Python binding. Nothing here falls back to a CPU implementation: if the
library is missing, using the API raises.
"""
from . import inputs  # noqa: F401  (seeded synthetic inputs, no method arithmetic)

__all__ = ["inputs", "api", "workloads"]


def __getattr__(name):
    if name in ("api", "workloads"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
