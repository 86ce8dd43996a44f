"""MI355X (gfx950) docking hot path: batched pose scoring and differential
evolution behind the C ABI of include/dock.h.

``paper_2509_12232_amd.dock`` is the binding (importing it requires the built
``libdock.so``); ``paper_2509_12232_amd.build`` compiles it with hipcc.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdock.so")
