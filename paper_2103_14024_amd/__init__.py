"""MI355X-native PlenOctree renderer (placeholder; filled in below)."""
