"""CPU reference of the hot path. TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from this package. The product path (the HIP
library and its binding) never imports, links or executes it, and this package
never imports the product path.
"""
