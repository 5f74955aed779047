"""EmbedSOM projection on AMD MI355X (gfx950).

The GPU library (``libesom.so``) is loaded lazily by ``paper_2201_00701_amd.esom``;
importing the package itself loads nothing.
"""
