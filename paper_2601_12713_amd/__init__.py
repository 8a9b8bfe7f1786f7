"""MI355X-native content digest and mapping-trace analysis (OMPDataPerf hot path)."""
__version__ = "0.1.0"
