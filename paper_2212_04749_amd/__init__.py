"""MI355X-native sliced multi-amplitude tensor-network contraction (ma-TNC).

Host side (pure Python, no GPU): ``circuit_tn`` builds the fused circuit
network, ``planner`` finds the contraction order and the sliced index set.
Device side: ``libmatnc.so`` (HIP, gfx950) behind the C ABI declared in
``include/matnc.h``; ``binding`` is the ctypes layer with the same names and
``api`` the convenience wrapper that passes torch device buffers and streams.
"""

__version__ = "0.1.0"
