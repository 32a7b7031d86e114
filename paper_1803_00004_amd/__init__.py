"""MI355X (gfx950) N-term bilateral filter: C-ABI library libbf.so + ctypes binding."""
from . import bf
from .bf import Plan, filter, filter_batch, workspace, BFError

__all__ = ["bf", "Plan", "filter", "filter_batch", "workspace", "BFError"]
