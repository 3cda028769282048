"""MI355X-native bi-directional pedestrian update (LEM and ACO) of
Dutta, McLeod and Friesen, arXiv 1412.4933.

Modules:
  pedsim     ctypes binding of the C ABI in include/pedsim.h (libpedsim.so)
  scenarios  seeded synthetic initial states
  build      hipcc build of libpedsim.so for gfx950
"""
__all__ = ["pedsim", "scenarios", "build"]
