"""MI355X-native k-bit LSB steganography (embed / extract) over gfx950 HIP."""
